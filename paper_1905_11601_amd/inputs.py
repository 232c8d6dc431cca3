"""Seeded synthetic inputs shared by the tests, the oracle and the benchmark.

This module holds none of the solver's arithmetic: it draws random numbers and
samples closed-form sine series at grid coordinates handed in by the caller
(as arrays), so both the HIP path and the CPU oracle can be fed bit-identical
inputs.  Everything is NumPy float64 with the PCG64 generator.

Storage convention (same as the library): a field has shape (nz+2, ny+2, nx+2),
index [k, j, i]; u lives on x-faces (i = 0..nx), v on y-faces, w on z-faces,
T at cell centres with one wall node per side.  A 4-field array is
(u, v, w, T).

Recipe of the synthetic base flow (the stand-in for a computed steady state):
* vector potential A = (Ax, Ay, Az), each a sum over l, m, n = 1..modes of
  c_lmn sin(l pi x) sin(m pi y) sin(n pi z), c ~ U(-1, 1) / (l^2 + m^2 + n^2),
  sampled on the cell edges of the staggered grid, wall edges forced to 0;
* U = discrete curl of A, so its discrete divergence vanishes and its wall
  normal components are zero; tangential wall nodes 0; scaled to max|U| = amp_u;
* Theta = (1 - x) + amp_t * (sine series of the same law, scaled to max-abs 1)
  at the cells; wall nodes from the inhomogeneous temperature conditions
  T = 1 - x on the x-, z- and conducting y-walls, copy of the adjacent value on
  insulated y-walls; edge nodes 0.
"""
import numpy as np

CC, AA = 0, 1


def _coef(rng, modes):
    l = np.arange(1, modes + 1)
    w = 1.0 / (l[:, None, None] ** 2 + l[None, :, None] ** 2 + l[None, None, :] ** 2)
    return rng.uniform(-1.0, 1.0, size=(modes, modes, modes)) * w


def _sines(x, modes):
    l = np.arange(1, modes + 1)
    return np.sin(np.pi * l[:, None] * np.asarray(x)[None, :])


def _series(C, x, y, z, modes):
    """sum_lmn C[l,m,n] sin(l pi x_i) sin(m pi y_j) sin(n pi z_k) as [k, j, i]."""
    return np.einsum('lmn,li,mj,nk->kji', C, _sines(x, modes), _sines(y, modes),
                     _sines(z, modes), optimize=True)


def conduction_state(c, span_bc):
    """U = 0, Theta = 1 - x at every cell and wall node (edges 0)."""
    cx, cy, cz = c
    nx, ny, nz = len(cx) - 2, len(cy) - 2, len(cz) - 2
    out = np.zeros((4, nz + 2, ny + 2, nx + 2))
    out[3] = _theta_walls(np.broadcast_to(1.0 - cx, (nz + 2, ny + 2, nx + 2)).copy(),
                          cx, span_bc)
    return out


def _theta_walls(T, cx, span_bc):
    nz, ny, nx = T.shape[0] - 2, T.shape[1] - 2, T.shape[2] - 2
    lin = 1.0 - cx                                   # 1 at x=0, 0 at x=1
    T[1:nz + 1, 1:ny + 1, 0] = lin[0]
    T[1:nz + 1, 1:ny + 1, nx + 1] = lin[nx + 1]
    T[0, 1:ny + 1, 1:nx + 1] = lin[None, 1:nx + 1]
    T[nz + 1, 1:ny + 1, 1:nx + 1] = lin[None, 1:nx + 1]
    if span_bc == CC:
        T[1:nz + 1, 0, 1:nx + 1] = lin[None, 1:nx + 1]
        T[1:nz + 1, ny + 1, 1:nx + 1] = lin[None, 1:nx + 1]
    else:
        T[1:nz + 1, 0, 1:nx + 1] = T[1:nz + 1, 1, 1:nx + 1]
        T[1:nz + 1, ny + 1, 1:nx + 1] = T[1:nz + 1, ny, 1:nx + 1]
    # edges and corners of the wall layers are never read by the stencils
    for sl in _edges(nx, ny, nz):
        T[sl] = 0.0
    return T


def _edges(nx, ny, nz):
    out = []
    for kk in (0, nz + 1):
        for jj in (0, ny + 1):
            out.append((kk, jj, slice(None)))
        for ii in (0, nx + 1):
            out.append((kk, slice(None), ii))
    for jj in (0, ny + 1):
        for ii in (0, nx + 1):
            out.append((slice(None), jj, ii))
    return out


def synthetic_base(f, c, h, span_bc, seed_u=1905, seed_t=1906, modes=8,
                   amp_u=0.1, amp_t=0.05):
    """Divergence-free synthetic base flow (U, V, W, Theta); see module doc.

    f, c, h: per-axis tuples of face coordinates f[0..n], centres c[0..n+1]
    (wall nodes included) and widths h[0..n+1] (h[i] = f[i] - f[i-1])."""
    fx, fy, fz = f
    cx, cy, cz = c
    hx, hy, hz = h
    nx, ny, nz = len(fx) - 1, len(fy) - 1, len(fz) - 1
    rng = np.random.default_rng(seed_u)
    Cx, Cy, Cz = _coef(rng, modes), _coef(rng, modes), _coef(rng, modes)
    # edge-sampled potential components (index [k, j, i] of the edge)
    Ax = _series(Cx, cx[1:nx + 1], fy, fz, modes)    # (nz+1, ny+1, nx)  i=1..nx
    Ay = _series(Cy, fx, cy[1:ny + 1], fz, modes)    # (nz+1, ny, nx+1)  j=1..ny
    Az = _series(Cz, fx, fy, cz[1:nz + 1], modes)    # (nz, ny+1, nx+1)  k=1..nz
    Ax[:, [0, ny], :] = 0.0
    Ax[[0, nz], :, :] = 0.0
    Ay[:, :, [0, nx]] = 0.0
    Ay[[0, nz], :, :] = 0.0
    Az[:, :, [0, nx]] = 0.0
    Az[:, [0, ny], :] = 0.0
    out = np.zeros((4, nz + 2, ny + 2, nx + 2))
    hyj = hy[1:ny + 1][None, :, None]
    hzk = hz[1:nz + 1][:, None, None]
    hxi = hx[1:nx + 1][None, None, :]
    # u on x-faces i = 0..nx, j = 1..ny, k = 1..nz
    out[0, 1:nz + 1, 1:ny + 1, 0:nx + 1] = ((Az[:, 1:, :] - Az[:, :-1, :]) / hyj
                                            - (Ay[1:, :, :] - Ay[:-1, :, :]) / hzk)
    # v on y-faces j = 0..ny, i = 1..nx, k = 1..nz
    out[1, 1:nz + 1, 0:ny + 1, 1:nx + 1] = ((Ax[1:, :, :] - Ax[:-1, :, :]) / hzk
                                            - (Az[:, :, 1:] - Az[:, :, :-1]) / hxi)
    # w on z-faces k = 0..nz, i = 1..nx, j = 1..ny
    out[2, 0:nz + 1, 1:ny + 1, 1:nx + 1] = ((Ay[:, :, 1:] - Ay[:, :, :-1]) / hxi
                                            - (Ax[:, 1:, :] - Ax[:, :-1, :]) / hyj)
    out[:3] *= amp_u / np.abs(out[:3]).max()
    rng = np.random.default_rng(seed_t)
    P = _series(_coef(rng, modes), cx[1:nx + 1], cy[1:ny + 1], cz[1:nz + 1], modes)
    T = np.zeros((nz + 2, ny + 2, nx + 2))
    T[1:nz + 1, 1:ny + 1, 1:nx + 1] = ((1.0 - cx[1:nx + 1])[None, None, :]
                                       + amp_t * P / np.abs(P).max())
    out[3] = _theta_walls(T, cx, span_bc)
    return out


def random_fields(n, seed):
    """i.i.d. N(0, 1) in all four stored fields (walls and padding included);
    the caller projects and normalises."""
    nx, ny, nz = n
    return np.random.default_rng(seed).standard_normal((4, nz + 2, ny + 2, nx + 2))


def random_pairs(n, count, seed_x=3000, seed_y=4000):
    return [(random_fields(n, seed_x + q), random_fields(n, seed_y + q)) for q in range(count)]
