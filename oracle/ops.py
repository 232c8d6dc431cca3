"""Oracle finite-volume operators (TEST INFRASTRUCTURE ONLY).

Plain PyTorch CPU float64, written from the discretisation reading of
Sec. 3.1 (second-order central MAC scheme in conservative flux form, linear
interpolation on the stretched grid, wall nodes stored).  Every operator
writes only interior rows; all other stored entries of its output are zero.

Storage (all fields share the padded shape (nz+2, ny+2, nx+2), index [k,j,i]):
  u : x-faces f_x[i] (i = 0..nx; i = nx+1 unused), centres c_y[j], c_z[k]
  v : y-faces, w : z-faces (cyclically)
  T : centres, wall nodes at i,j,k = 0 and n+1
A vector / base flow is a (4, nz+2, ny+2, nx+2) tensor: u, v, w, T (or U, V,
W, Theta).  Cell arrays (divergence, pressure) are compact (nz, ny, nx).

Contents and what pins each (see tests/test_oracle_*.py):
  adv_T, lap_T            energy flux divergence / Laplacian at cells
                          -- second-order convergence to (a.grad)b and
                             Laplacian of analytic fields; exact on linear T
  adv_mom, lap_mom        momentum at interior faces of one component
                          -- same convergence pins per component
  residual                steady residual of eqs (1)-(2) (pressure omitted)
                          -- conduction state F_T(0, 1-x) = 0, viscous-scaling
                             F = 0 at b = 0
  jacvec                  Jacobian of ``residual``, eqs (8)-(9)
                          -- [F(U+x) - F(U-x)]/2 = J(U) x exactly (F quadratic)
  div, grad               D (faces -> cells) and G (cells -> interior faces)
                          -- D G equals the Kronecker Laplacian of eq. (14)
"""
import torch

DT = torch.float64


def _off(a, s=1):
    o = [0, 0, 0]
    o[a] = s
    return tuple(o)


def _plus(p, q):
    return tuple(x + y for x, y in zip(p, q))


class Region:
    """Box of interior rows lo..hi (inclusive, (i,j,k) order) of a stored array."""

    def __init__(self, lo, hi):
        self.lo, self.hi = tuple(lo), tuple(hi)

    def idx(self, o=(0, 0, 0)):
        lo, hi = self.lo, self.hi
        return (slice(lo[2] + o[2], hi[2] + 1 + o[2]),
                slice(lo[1] + o[1], hi[1] + 1 + o[1]),
                slice(lo[0] + o[0], hi[0] + 1 + o[0]))

    def v(self, arr, o=(0, 0, 0)):
        return arr[self.idx(o)]

    def coef(self, vec, a, shift=0):
        """Grid vector ``vec`` (indexed by the natural index of axis a) over the
        region's index range on that axis, shaped to broadcast along a."""
        t = torch.as_tensor(vec[self.lo[a] + shift:self.hi[a] + 1 + shift], dtype=DT)
        shape = [1, 1, 1]
        shape[2 - a] = -1
        return t.reshape(shape)


def cells(grid):
    return Region((1, 1, 1), grid.n)


def faces(grid, a):
    hi = list(grid.n)
    hi[a] -= 1
    return Region((1, 1, 1), hi)


# --------------------------------------------------------------------------
# energy equation, eq. (1) / (8): rows at cells
# --------------------------------------------------------------------------

def adv_T(grid, a, b, axes=(0, 1, 2)):
    """sum over axes of [a_n b_face]_{face-}^{face+} / h : flux form of (a.grad) b.

    a: three velocity fields (staggered normal components), b: cell field;
    ``axes`` restricts the sum (the term a_al d b / d x_al of each axis al)."""
    R = cells(grid)
    out = 0.0
    for al in axes:
        g = grid.ax[al]
        wp, wm = R.coef(g.w, al, 0), R.coef(g.w, al, -1)
        hh = R.coef(g.h, al, 0)
        e, em = _off(al, 1), _off(al, -1)
        b_plus = (1 - wp) * R.v(b) + wp * R.v(b, e)
        b_minus = (1 - wm) * R.v(b, em) + wm * R.v(b)
        out = out + (R.v(a[al]) * b_plus - R.v(a[al], em) * b_minus) / hh
    return out


def lap_T(grid, b):
    R = cells(grid)
    out = 0.0
    for al in range(3):
        g = grid.ax[al]
        dp, dm, hh = R.coef(g.d, al, 0), R.coef(g.d, al, -1), R.coef(g.h, al, 0)
        e, em = _off(al, 1), _off(al, -1)
        out = out + ((R.v(b, e) - R.v(b)) / dp - (R.v(b) - R.v(b, em)) / dm) / hh
    return out


# --------------------------------------------------------------------------
# momentum equation, eq. (2) / (9): rows at interior faces normal to axis al
# --------------------------------------------------------------------------

def adv_mom(grid, al, a, b):
    """Flux form of (a.grad) b for the velocity component al (b = that component
    of the transported field), on the control volume around the al-face.

    Normal direction: averages of the two faces to the cell centres (exact
    midpoints).  Tangential direction be: the transporting component a_be is
    interpolated along al to the face position f_al[i] with w_al[i], the
    transported b is interpolated along be to the edge f_be[j] with w_be[j]."""
    R = faces(grid, al)
    g = grid.ax[al]
    e, em = _off(al, 1), _off(al, -1)
    dd = R.coef(g.d, al, 0)
    A_p = 0.5 * (R.v(a[al]) + R.v(a[al], e))
    B_p = 0.5 * (R.v(b) + R.v(b, e))
    A_m = 0.5 * (R.v(a[al], em) + R.v(a[al]))
    B_m = 0.5 * (R.v(b, em) + R.v(b))
    out = (A_p * B_p - A_m * B_m) / dd
    wa = R.coef(g.w, al, 0)
    for be in range(3):
        if be == al:
            continue
        gb = grid.ax[be]
        f, fm = _off(be, 1), _off(be, -1)
        wbp, wbm = R.coef(gb.w, be, 0), R.coef(gb.w, be, -1)
        hb = R.coef(gb.h, be, 0)
        At_p = (1 - wa) * R.v(a[be]) + wa * R.v(a[be], e)
        Bt_p = (1 - wbp) * R.v(b) + wbp * R.v(b, f)
        At_m = (1 - wa) * R.v(a[be], fm) + wa * R.v(a[be], _plus(e, fm))
        Bt_m = (1 - wbm) * R.v(b, fm) + wbm * R.v(b)
        out = out + (At_p * Bt_p - At_m * Bt_m) / hb
    return out


def lap_mom(grid, al, b):
    R = faces(grid, al)
    g = grid.ax[al]
    e, em = _off(al, 1), _off(al, -1)
    hp, hm, dd = R.coef(g.h, al, 1), R.coef(g.h, al, 0), R.coef(g.d, al, 0)
    out = ((R.v(b, e) - R.v(b)) / hp - (R.v(b) - R.v(b, em)) / hm) / dd
    for be in range(3):
        if be == al:
            continue
        gb = grid.ax[be]
        f, fm = _off(be, 1), _off(be, -1)
        dp, dm, hb = R.coef(gb.d, be, 0), R.coef(gb.d, be, -1), R.coef(gb.h, be, 0)
        out = out + ((R.v(b, f) - R.v(b)) / dp - (R.v(b) - R.v(b, fm)) / dm) / hb
    return out


def buoyancy(grid, T):
    """T interpolated to the interior z-faces (the T e_z term of eq. (2))."""
    R = faces(grid, 2)
    wz = R.coef(grid.ax[2].w, 2, 0)
    return (1 - wz) * R.v(T) + wz * R.v(T, _off(2, 1))


# --------------------------------------------------------------------------
# residual and Jacobian
# --------------------------------------------------------------------------

class Params:
    """nu = Gr^-1/2, kappa = nu/Pr, buoyancy coefficient b = 1 (eqs (1)-(2))."""

    def __init__(self, Gr, Pr, nu=None, kappa=None, b=1.0):
        self.Gr, self.Pr = Gr, Pr
        self.nu = Gr ** -0.5 if nu is None else nu
        self.kappa = self.nu / Pr if kappa is None else kappa
        self.b = b


def residual(grid, prm, base):
    """F(U, Theta) of the steady eqs (1)-(2) at interior rows, pressure omitted."""
    U = [base[0], base[1], base[2]]
    Th = base[3]
    out = torch.zeros_like(base)
    for al in range(3):
        R = faces(grid, al)
        r = prm.nu * lap_mom(grid, al, U[al]) - adv_mom(grid, al, U, U[al])
        if al == 2:
            r = r + prm.b * buoyancy(grid, Th)
        out[al][R.idx()] = r
    R = cells(grid)
    out[3][R.idx()] = prm.kappa * lap_T(grid, Th) - adv_T(grid, U, Th)
    return out


# Coupling terms of the linearised eqs (8)-(9) that the mechanism experiment
# of Sec. 4.2 switches off one at a time (bit i of a term mask):
TERM_BUOYANCY = 0      # T e_z in the momentum rows
TERM_U_GRAD_V = 1      # (U.grad) v in the momentum rows
TERM_V_GRAD_U = 2      # (v.grad) U in the momentum rows
TERM_U_GRAD_T = 3      # U_a dT/dx_a in the energy rows, bits 3, 4, 5 for a = x, y, z
TERM_V_GRAD_TH = 6     # v_a dTheta/dx_a in the energy rows, bits 6, 7, 8
ALL_TERMS = (1 << 9) - 1


def jacvec(grid, prm, base, x, terms=ALL_TERMS):
    """J(U, Theta) x, the linearisation of ``residual`` about the base flow:
    velocity rows  nu Lap v - (U.grad) v - (v.grad) U + T e_z      (eq. 9)
    energy rows    kappa Lap T - (U.grad) T - (v.grad) Theta        (eq. 8)
    ``terms``: bit mask of the coupling terms kept (TERM_*; the viscous and
    conductive terms are always kept).
    """
    def on(bit):
        return bool(terms >> bit & 1)

    U = [base[0], base[1], base[2]]
    Th = base[3]
    v = [x[0], x[1], x[2]]
    T = x[3]
    out = torch.zeros_like(x)
    for al in range(3):
        R = faces(grid, al)
        r = prm.nu * lap_mom(grid, al, v[al])
        if on(TERM_U_GRAD_V):
            r = r - adv_mom(grid, al, U, v[al])
        if on(TERM_V_GRAD_U):
            r = r - adv_mom(grid, al, v, U[al])
        if al == 2 and on(TERM_BUOYANCY):
            r = r + prm.b * buoyancy(grid, T)
        out[al][R.idx()] = r
    R = cells(grid)
    e = prm.kappa * lap_T(grid, T)
    ax_u = tuple(a for a in range(3) if on(TERM_U_GRAD_T + a))
    ax_v = tuple(a for a in range(3) if on(TERM_V_GRAD_TH + a))
    if ax_u:
        e = e - adv_T(grid, U, T, ax_u)
    if ax_v:
        e = e - adv_T(grid, v, Th, ax_v)
    out[3][R.idx()] = e
    return out


# --------------------------------------------------------------------------
# divergence and gradient (SIMPLE steps 1-2)
# --------------------------------------------------------------------------

def div(grid, vel):
    """D v at cells, compact (nz, ny, nx): sum over axes (face+ - face-)/h."""
    R = cells(grid)
    out = 0.0
    for al in range(3):
        hh = R.coef(grid.ax[al].h, al, 0)
        out = out + (R.v(vel[al]) - R.v(vel[al], _off(al, -1))) / hh
    return out


def grad(grid, phi):
    """G phi on interior faces (zero on wall faces: Neumann condition of the
    pressure correction), returned as three stored face fields."""
    full = torch.zeros(grid.shape, dtype=DT)
    full[cells(grid).idx()] = phi
    out = []
    for al in range(3):
        R = faces(grid, al)
        g = torch.zeros(grid.shape, dtype=DT)
        dd = R.coef(grid.ax[al].d, al, 0)
        g[R.idx()] = (R.v(full, _off(al, 1)) - R.v(full)) / dd
        out.append(g)
    return out
