"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
function that include/fvk.h declares, and its host eigen-solver used for
eq. (15) agrees with LAPACK."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1905_11601_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fvk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, re.M))
                  - {"typedef"})


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_null_and_bad_arguments_return_einval():
    lib = _lib.load()
    assert lib.fvk_destroy(None) == 1
    assert lib.fvk_layout(None, None, None, None) == 1
    h = ctypes.c_void_p()
    # invalid sizes / enums are rejected before any device call
    assert lib.fvk_create(ctypes.byref(h), 1, 8, 8, 0, 0.0, 0, 1e5, 0.71, 0, None) == 1
    assert lib.fvk_create(ctypes.byref(h), 8, 8, 8, 7, 0.0, 0, 1e5, 0.71, 0, None) == 1
    assert lib.fvk_create(ctypes.byref(h), 8, 8, 8, 0, 0.0, 3, 1e5, 0.71, 0, None) == 1
    assert lib.fvk_create(ctypes.byref(h), 8, 8, 8, 1, 0.5, 0, 1e5, 0.71, 0, None) == 1
    assert lib.fvk_create(ctypes.byref(h), 8, 8, 8, 0, 0.0, 0, -1.0, 0.71, 0, None) == 1
    assert h.value is None


@pytest.mark.parametrize("n", [1, 2, 7, 64, 257])
def test_tridiag_eig_matches_lapack(n):
    from paper_1905_11601_amd import tridiag_eig
    rng = np.random.default_rng(n)
    d = rng.standard_normal(n) * 3
    e = rng.standard_normal(max(n - 1, 1))[: n - 1] if n > 1 else np.zeros(1)
    lam, Q = tridiag_eig(d, e if n > 1 else np.zeros(1))
    T = np.diag(d) + (np.diag(e, 1) + np.diag(e, -1) if n > 1 else 0)
    ref = np.linalg.eigvalsh(T)
    assert np.max(np.abs(np.sort(lam) - ref)) < 1e-12 * max(1, np.abs(ref).max())
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) < 1e-12
    assert np.max(np.abs(T @ Q - Q * lam[None, :])) < 1e-11 * max(1, np.abs(ref).max())


def test_tridiag_eig_on_stretched_neumann_operator():
    # the set-up case itself: V^1/2 Dxx V^-1/2 on a 256-cell tanh grid, whose
    # eigenvalues span 0 .. ~ -4/h_min^2
    from oracle.grid import Grid, TANH
    from oracle.tpf import neumann_1d
    from paper_1905_11601_amd import tridiag_eig
    ax = Grid(256, kind=TANH, s=1.5).ax[0]
    A = neumann_1d(ax)
    vh = np.sqrt(ax.h[1:-1])
    S = (vh[:, None] * A) / vh[None, :]
    lam, Q = tridiag_eig(np.diag(S).copy(), np.diag(S, 1).copy())
    ref = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert np.max(np.abs(np.sort(lam) - ref)) < 1e-12 * np.abs(ref).max()
    assert np.max(np.abs(Q.T @ Q - np.eye(256))) < 1e-12
