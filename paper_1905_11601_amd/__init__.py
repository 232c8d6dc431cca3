"""fvk: Krylov-vector engine for the Newton / Arnoldi stability solver of
buoyancy convection in a laterally heated cube (Gelfgat, arXiv:1905.11601) on
AMD Instinct MI355X.

Python binding over the C-ABI library ``libfvk.so`` (declared in
``include/fvk.h``).  PyTorch supplies device memory and the stream; every
step of the computation runs in the library's HIP kernels.  The names follow
the C ABI: ``Ctx.fv_residual``, ``Ctx.fv_jacvec``, ``Ctx.simple_krylov_vec``,
``Ctx.arnoldi_step``, ``Ctx.newton_step``.

``paper_1905_11601_amd.inputs`` (seeded synthetic inputs) does not load the
library; everything else does, and fails loudly if it is missing.
"""
import ctypes

import numpy as np

CC, AA = 0, 1
UNIFORM, SINE, TANH = 0, 1, 2
FP64, MIXED = 0, 1
TPF_AUTO, TPF_AXES, TPF_PLANES = 0, 1, 2
# coupling terms of the linearised operator (fvk_set_terms bit masks)
TERM_BUOYANCY, TERM_U_GRAD_V, TERM_V_GRAD_U = 1, 2, 4
TERM_U_GRAD_T = (8, 16, 32)        # U dT/dx, V dT/dy, W dT/dz
TERM_V_GRAD_TH = (64, 128, 256)    # u dTheta/dx, v dTheta/dy, w dTheta/dz
TERMS_ALL = 511


class FvkError(RuntimeError):
    def __init__(self, status, msg):
        from ._lib import STATUS
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Ctx:
    """One grid / parameter set on one device stream (see fvk_create)."""

    def __init__(self, nx, ny=None, nz=None, grid=TANH, s=1.5, span_bc=CC, Gr=1e6, Pr=0.71,
                 prec=FP64, device="cuda:0", stream=None):
        import torch
        from . import _lib
        self.lib = _lib.load()
        self.torch = torch
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.n = (nx, ny, nz)
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.fvk_create(ctypes.byref(h), nx, ny, nz, grid, float(s), span_bc,
                                 float(Gr), float(Pr), prec, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise FvkError(st, "fvk_create failed")
        self.h = h
        self.span_bc, self.grid_kind, self.s = span_bc, grid, s
        self.Gr, self.Pr, self.prec = Gr, Pr, prec
        self.terms = TERMS_ALL
        self.shift = 0.0
        F = ctypes.c_size_t()
        N = ctypes.c_size_t()
        self.lib.fvk_layout(h, None, ctypes.byref(F), ctypes.byref(N))
        self.F, self.N = F.value, N.value
        self.shape4 = (4, nz + 2, ny + 2, nx + 2)

    # ---- housekeeping ------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.fvk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise FvkError(st, self.lib.fvk_last_error(self.h).decode())

    def _vec(self, t, name):
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda
                and t.is_contiguous() and t.numel() == self.N):
            raise ValueError(f"{name}: need a contiguous float64 CUDA tensor of {self.N} elements")
        return _ptr(t)

    def empty(self):
        return self.torch.empty(self.shape4, dtype=self.torch.float64, device=self.device)

    def zeros(self):
        return self.torch.zeros(self.shape4, dtype=self.torch.float64, device=self.device)

    def set_params(self, Gr, Pr=None):
        Pr = self.Pr if Pr is None else Pr
        self._check(self.lib.fvk_set_params(self.h, float(Gr), float(Pr)))
        self.Gr, self.Pr = Gr, Pr

    def set_coeffs(self, nu, kappa, b):
        self._check(self.lib.fvk_set_coeffs(self.h, float(nu), float(kappa), float(b)))

    def set_terms(self, mask=TERMS_ALL):
        """Coupling terms kept in the linearised operator (TERM_* bits)."""
        self._check(self.lib.fvk_set_terms(self.h, int(mask)))
        self.terms = int(mask)

    def set_shift(self, sigma):
        """Krylov operator A + sigma P in simple_krylov_vec / arnoldi_step
        (fvk_set_shift); 0 restores A."""
        self._check(self.lib.fvk_set_shift(self.h, float(sigma)))
        self.shift = float(sigma)

    def set_precision(self, prec):
        self._check(self.lib.fvk_set_precision(self.h, prec))
        self.prec = prec

    def set_tpf_path(self, path):
        """Kernels of the TPF solve (fvk_set_tpf_path): TPF_AUTO (= TPF_AXES),
        TPF_AXES (one launch per axis transform) or TPF_PLANES (three plane
        launches, axes of 4 .. 128 cells; measured slower, opt-in)."""
        self._check(self.lib.fvk_set_tpf_path(self.h, int(path)))

    def tpf_path(self):
        """TPF_AXES or TPF_PLANES: the kernels the solve runs."""
        v = ctypes.c_int()
        self._check(self.lib.fvk_get_tpf_path(self.h, ctypes.byref(v)))
        return v.value

    def set_simple(self, tol, max_passes):
        self._check(self.lib.fvk_set_simple(self.h, float(tol), int(max_passes)))

    def axis(self, a):
        n = self.n[a]
        f = np.zeros(n + 1)
        c = np.zeros(n + 2)
        h = np.zeros(n + 2)
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.fvk_grid_axis(self.h, a, f.ctypes.data_as(dp), c.ctypes.data_as(dp),
                                           h.ctypes.data_as(dp)))
        return f, c, h

    def coords(self):
        ax = [self.axis(a) for a in range(3)]
        return tuple(a[0] for a in ax), tuple(a[1] for a in ax), tuple(a[2] for a in ax)

    # ---- operators (C-ABI names) ------------------------------------------
    def fv_residual(self, base, out=None, project=False):
        out = self.empty() if out is None else out
        self._check(self.lib.fv_residual(self.h, self._vec(base, "base"), self._vec(out, "F"),
                                         int(bool(project))))
        return out

    def fv_jacvec(self, base, x, out=None, transpose=False):
        out = self.empty() if out is None else out
        self._check(self.lib.fv_jacvec(self.h, self._vec(base, "base"), self._vec(x, "x"),
                                       self._vec(out, "y"), int(bool(transpose))))
        return out

    def project(self, x, out=None, transpose=False):
        out = self.empty() if out is None else out
        self._check(self.lib.fvk_project(self.h, self._vec(x, "x"), self._vec(out, "y"),
                                         int(bool(transpose))))
        return out

    def simple_krylov_vec(self, base, x, out=None, transpose=False, p_out=None, info=False):
        out = self.empty() if out is None else out
        pp = None
        if p_out is not None:
            if p_out.numel() != self.n[0] * self.n[1] * self.n[2] or p_out.dtype != self.torch.float64:
                raise ValueError("p_out: need nx*ny*nz float64")
            pp = _ptr(p_out)
        if info:
            k = ctypes.c_int()
            d = ctypes.c_double()
            st = self.lib.simple_krylov_vec(self.h, self._vec(base, "base"), self._vec(x, "x"),
                                            self._vec(out, "y"), pp, int(bool(transpose)),
                                            ctypes.byref(k), ctypes.byref(d))
            self._check(st)
            return out, k.value, d.value
        self._check(self.lib.simple_krylov_vec(self.h, self._vec(base, "base"), self._vec(x, "x"),
                                               self._vec(out, "y"), pp, int(bool(transpose)),
                                               None, None))
        return out

    def psi_projection(self, vel, axis):
        """(vproj, psi) for the planes normal to `axis` (fvk_psi_projection):
        vproj a (3, nz+2, ny+2, nx+2) tensor, psi one stored field.  vel: a
        4-field vector (or 3 velocity fields) on the device."""
        torch = self.torch
        if not (isinstance(vel, torch.Tensor) and vel.dtype == torch.float64 and vel.is_cuda
                and vel.is_contiguous() and vel.numel() in (self.N, 3 * self.F)):
            raise ValueError("vel: contiguous float64 CUDA tensor of 3 or 4 fields")
        vp = torch.empty((3,) + self.shape4[1:], dtype=torch.float64, device=self.device)
        psi = torch.empty(self.shape4[1:], dtype=torch.float64, device=self.device)
        self._check(self.lib.fvk_psi_projection(self.h, _ptr(vel), int(axis), _ptr(vp), _ptr(psi)))
        return vp, psi

    def simple_stats(self):
        d = ctypes.c_double()
        k = ctypes.c_int()
        self._check(self.lib.fvk_simple_stats(self.h, ctypes.byref(d), ctypes.byref(k)))
        return d.value, k.value

    def mixed_passes(self):
        """(fixed pass count of asynchronous mixed calls, calibrated?)"""
        k = ctypes.c_int()
        c = ctypes.c_int()
        self._check(self.lib.fvk_mixed_passes(self.h, ctypes.byref(k), ctypes.byref(c)))
        return k.value, bool(c.value)

    STAGES = ("jacvec", "div", "transform", "correct", "ortho")

    def set_timing(self, stages=()):
        mask = 0
        for s_ in stages:
            mask |= 1 << self.STAGES.index(s_)
        self._check(self.lib.fvk_set_timing(self.h, mask))

    def timing_read(self):
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int * 5)()
        self._check(self.lib.fvk_timing_read(self.h, ms, cnt))
        return {s_: (ms[q], cnt[q]) for q, s_ in enumerate(self.STAGES)}

    def arnoldi_step(self, base, V, j, transpose=False):
        """V: (m+1, N) float64 CUDA tensor (rows are basis vectors)."""
        if V.dim() != 2 or V.shape[1] != self.N or not V.is_contiguous() or j + 1 >= V.shape[0]:
            raise ValueError("V must be a contiguous (m+1, N) tensor with room for vector j+1")
        h = np.zeros(j + 2)
        st = self.lib.arnoldi_step(self.h, self._vec(base, "base"), _ptr(V), V.shape[1], j,
                                   h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   int(bool(transpose)))
        if st not in (0, 5):
            self._check(st)
        return h, st == 5

    def _hess(self, H):
        if not (isinstance(H, np.ndarray) and H.dtype == np.float64 and H.ndim == 2
                and H.flags.c_contiguous):
            raise ValueError("H must be a C-contiguous float64 (rows, cols) array")
        return H.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def arnoldi_step_lagged(self, base, V, j, H, transpose=False):
        """Lagged-CGS2 Arnoldi step j (see include/fvk.h): V (m+1, N) CUDA
        tensor, H host (rows >= j+2, cols >= j+1) updated in place."""
        if V.dim() != 2 or V.shape[1] != self.N or not V.is_contiguous() or j + 1 >= V.shape[0]:
            raise ValueError("V must be a contiguous (m+1, N) tensor with room for vector j+1")
        if H.shape[0] < j + 2 or H.shape[1] < j + 1:
            raise ValueError("H too small for step j")
        self._check(self.lib.arnoldi_step_lagged(self.h, self._vec(base, "base"), _ptr(V),
                                                 V.shape[1], j, self._hess(H), H.shape[1],
                                                 int(bool(transpose))))

    def arnoldi_step_lagged_applied(self, V, j, H):
        """Lagged-CGS2 step j for an operator applied by the caller: V[j+1]
        already holds it applied to V[j]."""
        if V.dim() != 2 or V.shape[1] != self.N or not V.is_contiguous() or j + 1 >= V.shape[0]:
            raise ValueError("V must be a contiguous (m+1, N) tensor with room for vector j+1")
        if H.shape[0] < j + 2 or H.shape[1] < j + 1:
            raise ValueError("H too small for step j")
        self._check(self.lib.arnoldi_step_lagged_applied(self.h, _ptr(V), V.shape[1], j,
                                                         self._hess(H), H.shape[1]))

    def lincomb3(self, z, a, x, b, y, c):
        """z <- a x + b y + c z (library kernel, no host transfer)."""
        if not (z.numel() == x.numel() == y.numel()) or not all(
                t.is_contiguous() for t in (x, y, z)):
            raise ValueError("lincomb3: contiguous tensors of equal size")
        self._check(self.lib.fvk_lincomb3(self.h, _ptr(z), float(a), _ptr(x), float(b), _ptr(y),
                                          float(c), z.numel()))
        return z

    def arnoldi_finish(self, V, j, H):
        """Completes a lagged sequence: slot j becomes the unit vector v_j."""
        if V.dim() != 2 or V.shape[1] != self.N or not V.is_contiguous() or j >= V.shape[0]:
            raise ValueError("V must be a contiguous (m+1, N) tensor with a slot j")
        if H.shape[0] < j + 1 or (j > 0 and H.shape[1] < j):
            raise ValueError("H too small")
        self._check(self.lib.arnoldi_finish(self.h, _ptr(V), V.shape[1], j, self._hess(H),
                                            max(H.shape[1], 1)))

    def multidot(self, V, m, w):
        out = np.zeros(m)
        self._check(self.lib.fvk_multidot(self.h, _ptr(V), V.shape[-1], m, _ptr(w), self.N,
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def multidot_noalloc(self, V, m, w, out, n=None):
        """out[:m] <- V[:m] . w on the device, no allocation, no sync
        (fvk_multidot_noalloc); n defaults to the vector length."""
        n = self.N if n is None else int(n)
        if not (out.is_cuda and out.dtype == self.torch.float64 and out.numel() >= m):
            raise ValueError("out: float64 CUDA tensor with at least m entries")
        self._check(self.lib.fvk_multidot_noalloc(self.h, _ptr(V), V.shape[-1], m, _ptr(w), n,
                                                  _ptr(out)))
        return out

    def dot(self, x, y):
        return float(self.multidot(x.reshape(1, -1), 1, y)[0])

    def multiaxpy(self, w, alpha, V, c):
        c = np.ascontiguousarray(c, dtype=np.float64)
        self._check(self.lib.fvk_multiaxpy(self.h, _ptr(w), float(alpha), _ptr(V), V.shape[-1],
                                           len(c), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           self.N))

    def axpby(self, y, a, x, b):
        """y <- a x + b y (library kernel); x may be y (scaling)."""
        if y.numel() != x.numel() or not (y.is_contiguous() and x.is_contiguous()):
            raise ValueError("axpby: contiguous tensors of equal size")
        self._check(self.lib.fvk_axpby(self.h, _ptr(y), float(a), _ptr(x), float(b), y.numel()))
        return y

    def normalize(self, x):
        nrm = self.dot(x, x) ** 0.5
        self.axpby(x, 1.0 / nrm, x, 0.0)
        return nrm

    def basis_rotate(self, V, Q):
        """V[:k] <- (V[:m]^T Q)^T with Q (m, k) real."""
        Q = np.asfortranarray(Q, dtype=np.float64)
        m, k = Q.shape
        self._check(self.lib.fvk_basis_rotate(self.h, _ptr(V), V.shape[1], m,
                                              Q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              k, self.N))

    def _opts(self, opts):
        from ._lib import NewtonOpts
        o = NewtonOpts()
        self.lib.fvk_newton_defaults(ctypes.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        return o

    def linear_solve(self, base, b, x=None, **opts):
        """Solve A x = b (GMRES(m) then BiCGstab(2)); returns (x, report)."""
        from ._lib import NewtonReport
        x = self.zeros() if x is None else x
        o = self._opts(opts)
        r = NewtonReport()
        st = self.lib.fvk_linear_solve(self.h, self._vec(base, "base"), self._vec(b, "b"),
                                       self._vec(x, "x"), ctypes.byref(o), ctypes.byref(r))
        rep = {f: getattr(r, f) for f, _ in NewtonReport._fields_}
        rep["status"] = st
        return x, rep

    def newton_step(self, base, **opts):
        from ._lib import NewtonOpts, NewtonReport
        o = NewtonOpts()
        self.lib.fvk_newton_defaults(ctypes.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        r = NewtonReport()
        st = self.lib.newton_step(self.h, self._vec(base, "base"), ctypes.byref(o), ctypes.byref(r))
        rep = {f: getattr(r, f) for f, _ in NewtonReport._fields_}
        rep["status"] = st
        return rep


def tridiag_eig(diag, off):
    """Host symmetric tridiagonal eigensolver of the library (eq. (15) set-up)."""
    from . import _lib
    lib = _lib.load()
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.float64)
    n = len(diag)
    lam = np.zeros(n)
    Q = np.zeros((n, n))
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.fvk_tridiag_eig(n, diag.ctypes.data_as(dp), off.ctypes.data_as(dp),
                             lam.ctypes.data_as(dp), Q.ctypes.data_as(dp))
    if st != 0:
        raise FvkError(st, "fvk_tridiag_eig failed")
    return lam, Q
