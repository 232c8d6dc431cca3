// Finite-volume stencil kernels on the staggered grid with stored wall nodes
// (paper Sec. 3.1: residual of eqs (1)-(2), Jacobian of eqs (8)-(9), the
// divergence / gradient pair of the SIMPLE pass, the temperature projection of
// eq. (21) in its boundary-local form) and their Euclidean transposes.
//
// Field layout: (nz+2, ny+2, nx+2), x fastest.  A 4-field vector holds
// u (x-faces), v (y-faces), w (z-faces), T (centres) back to back.  Rows of the
// momentum equation for component A are the interior A-faces
// (1 <= i_A <= n_A - 1, 1 <= i_B <= n_B for B != A); rows of the energy
// equation are the interior cells.  Forward kernels write every stored entry
// (0 where the operator has no row).
#include <algorithm>
#include <type_traits>

#include "fvk_internal.h"
#include "xcd.h"

namespace fvk {

namespace {

constexpr int BX = 64, BY = 4;

// XCD-aware block order for the per-point kernels: hardware block b runs on
// XCD b % 8, so consecutive blocks (one z-plane) would spread every plane over
// all eight L2s; give each XCD a contiguous range of logical blocks instead,
// so the neighbouring planes a block reads sit in its own L2.
struct Blk {
    int x, y, z;
    long lin;   // logical linear index (unique per block)
};

__device__ __forceinline__ Blk xcd_block() {
    const int nbx = gridDim.x, nby = gridDim.y;
    const long nb = long(nbx) * nby * gridDim.z;
    const long b = (long(blockIdx.z) * nby + blockIdx.y) * nbx + blockIdx.x;
    const long lb = xcd_remap(b, nb);
    Blk r;
    r.lin = lb;
    r.x = int(lb % nbx);
    r.y = int((lb / nbx) % nby);
    r.z = int(lb / (long(nbx) * nby));
    return r;
}

__device__ __forceinline__ bool face_row(const Geo &g, int A, int i, int j, int k) {
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int B = 0; B < 3; ++B) {
        const int hi = (B == A) ? g.n[B] - 1 : g.n[B];
        if (idx[B] < 1 || idx[B] > hi) return false;
    }
    return true;
}

__device__ __forceinline__ bool cell_row(const Geo &g, int i, int j, int k) {
    return i >= 1 && i <= g.n[0] && j >= 1 && j <= g.n[1] && k >= 1 && k <= g.n[2];
}


__device__ __forceinline__ long pos(const Geo &g, int i, int j, int k) {
    return (long(k) * g.np[1] + j) * g.np[0] + i;
}

// ---------------------------------------------------------------- forward

// Momentum row of component A at stored position p (an interior A-face).
// Returns nu*Lap(X_A) - [N_A(a1, b1_A) + N_A(a2, b2_A)] * adv_scale
//         + bcoef * T interpolated to the z-face (A == 2).
// N_A(a, b): conservative flux form of (a.grad) b_A on the A-face control
// volume: normal fluxes at the two adjacent cell centres (midpoint averages),
// tangential fluxes at the edges (a_B interpolated along A with w_A, b_A
// interpolated along B with w_B).
template <int A>
__device__ __forceinline__ double mom_row(const Geo &g, const int *idx, long p,
                                          const double *const *a1, const double *const *b1,
                                          const double *const *a2, const double *const *b2,
                                          double adv_scale, const double *X, double nu,
                                          const double *T, double bcoef) {
    const long sA = g.s[A];
    const int ia = idx[A];
    const AxisDev &aA = g.ax[A];
    const double idA = aA.id[ia];
    double adv, lap;
    {
        const double A1p = 0.5 * (a1[A][p] + a1[A][p + sA]), A1m = 0.5 * (a1[A][p - sA] + a1[A][p]);
        const double B1p = 0.5 * (b1[A][p] + b1[A][p + sA]), B1m = 0.5 * (b1[A][p - sA] + b1[A][p]);
        const double A2p = 0.5 * (a2[A][p] + a2[A][p + sA]), A2m = 0.5 * (a2[A][p - sA] + a2[A][p]);
        const double B2p = 0.5 * (b2[A][p] + b2[A][p + sA]), B2m = 0.5 * (b2[A][p - sA] + b2[A][p]);
        adv = (A1p * B1p - A1m * B1m + A2p * B2p - A2m * B2m) * idA;
        lap = ((X[p + sA] - X[p]) * aA.ih[ia + 1] - (X[p] - X[p - sA]) * aA.ih[ia]) * idA;
    }
    const double wa = aA.w[ia];
#pragma unroll
    for (int t = 1; t <= 2; ++t) {
        const int Bt = (A + t) % 3;
        const long sB = g.s[Bt];
        const int jb = idx[Bt];
        const AxisDev &aB = g.ax[Bt];
        const double wbp = aB.w[jb], wbm = aB.w[jb - 1];
        // transporting component Bt at the edges (A-face, Bt-face jb / jb-1)
        const double t1p = (1.0 - wa) * a1[Bt][p] + wa * a1[Bt][p + sA];
        const double t1m = (1.0 - wa) * a1[Bt][p - sB] + wa * a1[Bt][p + sA - sB];
        const double t2p = (1.0 - wa) * a2[Bt][p] + wa * a2[Bt][p + sA];
        const double t2m = (1.0 - wa) * a2[Bt][p - sB] + wa * a2[Bt][p + sA - sB];
        // transported component A at the same edges
        const double s1p = (1.0 - wbp) * b1[A][p] + wbp * b1[A][p + sB];
        const double s1m = (1.0 - wbm) * b1[A][p - sB] + wbm * b1[A][p];
        const double s2p = (1.0 - wbp) * b2[A][p] + wbp * b2[A][p + sB];
        const double s2m = (1.0 - wbm) * b2[A][p - sB] + wbm * b2[A][p];
        adv += (t1p * s1p - t1m * s1m + t2p * s2p - t2m * s2m) * aB.ih[jb];
        lap += ((X[p + sB] - X[p]) * aB.id[jb] - (X[p] - X[p - sB]) * aB.id[jb - 1]) * aB.ih[jb];
    }
    double r = nu * lap - adv_scale * adv;
    if (A == 2) r += bcoef * ((1.0 - wa) * T[p] + wa * T[p + sA]);
    return r;
}

// Energy row at an interior cell p: kappa Lap(Tl) - N_T(a1, b1) - N_T(a2, b2);
// N_T(a, b) = sum_A [a_A b_face]_{face-}^{face+} / h_A.  a2 may be null.
__device__ __forceinline__ double energy_row(const Geo &g, const int *idx, long p,
                                             const double *const *a1, const double *b1,
                                             const double *const *a2, const double *b2,
                                             const double *Tl, double kappa) {
    double adv = 0.0, lap = 0.0;
#pragma unroll
    for (int A = 0; A < 3; ++A) {
        const long sA = g.s[A];
        const int ia = idx[A];
        const AxisDev &aA = g.ax[A];
        const double wp = aA.w[ia], wm = aA.w[ia - 1], ih = aA.ih[ia];
        const double f1p = (1.0 - wp) * b1[p] + wp * b1[p + sA];
        const double f1m = (1.0 - wm) * b1[p - sA] + wm * b1[p];
        double a = a1[A][p] * f1p - a1[A][p - sA] * f1m;
        if (a2) {
            const double f2p = (1.0 - wp) * b2[p] + wp * b2[p + sA];
            const double f2m = (1.0 - wm) * b2[p - sA] + wm * b2[p];
            a += a2[A][p] * f2p - a2[A][p - sA] * f2m;
        }
        adv += a * ih;
        lap += ((Tl[p + sA] - Tl[p]) * aA.id[ia] - (Tl[p] - Tl[p - sA]) * aA.id[ia - 1]) * ih;
    }
    return kappa * lap - adv;
}

// y = J(base) x on every stored entry (velocity part to yv, T part to yT).
// With span_aa set (insulated y-walls and the extension requested) the
// temperature part is returned extended by the homogeneous BCs: insulated
// y-wall nodes = adjacent interior value, i.e. Ext_T (J x)_T; Dirichlet wall
// nodes are 0 either way.
// mode 0: Jacobian; mode 1: residual F(base) (x ignored).
template <int MODE>
__global__ __launch_bounds__(BX *BY) void k_jac(Geo g, Coefs c, int span_aa,
                                                const double *__restrict__ base,
                                                const double *__restrict__ x,
                                                double *__restrict__ yv,
                                                double *__restrict__ yT) {
    const Blk B = xcd_block();
    const int i = B.x * BX + threadIdx.x;
    const int j = B.y * BY + threadIdx.y;
    const int k = B.z;
    if (i >= g.np[0] || j >= g.np[1] || k >= g.np[2]) return;
    const long F = g.F;
    const long p = pos(g, i, j, k);
    const int idx[3] = {i, j, k};
    const double *U[3] = {base, base + F, base + 2 * F};
    const double *Th = base + 3 * F;
    const double *X[3] = {x, x + F, x + 2 * F};
    const double *XT = x + 3 * F;
    double out[3];
#pragma unroll
    for (int A = 0; A < 3; ++A) out[A] = 0.0;
    if (face_row(g, 0, i, j, k))
        out[0] = (MODE == 0) ? mom_row<0>(g, idx, p, U, X, X, U, 1.0, X[0], c.nu, XT, c.b)
                             : mom_row<0>(g, idx, p, U, U, U, U, 0.5, U[0], c.nu, Th, c.b);
    if (face_row(g, 1, i, j, k))
        out[1] = (MODE == 0) ? mom_row<1>(g, idx, p, U, X, X, U, 1.0, X[1], c.nu, XT, c.b)
                             : mom_row<1>(g, idx, p, U, U, U, U, 0.5, U[1], c.nu, Th, c.b);
    if (face_row(g, 2, i, j, k))
        out[2] = (MODE == 0) ? mom_row<2>(g, idx, p, U, X, X, U, 1.0, X[2], c.nu, XT, c.b)
                             : mom_row<2>(g, idx, p, U, U, U, U, 0.5, U[2], c.nu, Th, c.b);
    yv[p] = out[0];
    yv[p + F] = out[1];
    yv[p + 2 * F] = out[2];
    // temperature (row or insulated-wall copy of the adjacent row)
    double t = 0.0;
    int jr = j;
    bool have = cell_row(g, i, j, k);
    if (!have && span_aa && i >= 1 && i <= g.n[0] && k >= 1 && k <= g.n[2]) {
        if (j == 0) { jr = 1; have = true; }
        if (j == g.n[1] + 1) { jr = g.n[1]; have = true; }
    }
    if (have) {
        const int idr[3] = {i, jr, k};
        const long pr = pos(g, i, jr, k);
        t = (MODE == 0) ? energy_row(g, idr, pr, U, XT, X, Th, XT, c.kappa)
                        : energy_row(g, idr, pr, U, Th, nullptr, nullptr, Th, c.kappa);
    }
    yT[p] = t;
}

// ---------------------------------------------------------------- forward, tiled
//
// The Krylov-path Jacobian: 2.5D blocking.  A block owns a TX x H tile of the
// interior (i, j) plane and marches in k over a chunk of planes; planes k-1,
// k, k+1 of all eight input fields (x: u v w T, base: U V W Theta) with a
// one-point halo in i and j sit in an LDS ring, so every global value is
// loaded once per block (halo aside) with coalesced row loads, and the ~70
// neighbour reads per point come from LDS.  Every stored entry of the output
// is written exactly once: the interior by its own thread, the wall layers by
// the threads next to them, the k = 0 and k = nz+1 planes by the first and last
// chunk.  Blocks are remapped so that each XCD (one L2) gets a contiguous range
// of tiles and reuses the halo rows of its neighbours.

constexpr int TX = 64, TWP = TX + 2, NF = 8;
// A tile of TX x H interior points: its plane with the one-point halo, the
// threads of its block and the staged entries per thread and field.
template <int H>
struct Tile {
    static constexpr int TY = H, THP = H + 2, PLANE = TWP * THP, NT = TX * H,
                         PER = (PLANE + NT - 1) / NT;
};

// The thread's own column (offset 0 in i and j) at planes k-1, k, k+1 is
// carried in registers along the k-march: each centre value is read from LDS
// once (when its plane is staged) instead of at every use, which halves the
// LDS reads per point.
template <int PL>
struct TileAcc {
    static constexpr int PLANE = PL;
    const double *s[3];   // planes k-1, k, k+1
    int c;                // LDS offset of this thread's centre point
    double cen[3][NF];    // centres of planes k-1, k, k+1
    template <int D0, int D1, int D2>
    __device__ __forceinline__ double at(int f) const {
        if (D0 == 0 && D1 == 0) return cen[D2 + 1][f];
        return s[D2 + 1][f * PLANE + c + D1 * TWP + D0];
    }
    // before the march: centres of the first two planes (staged in pm, p0)
    __device__ __forceinline__ void first_centres(const double *pm, const double *p0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cen[0][f] = pm[f * PLANE + c];
            cen[1][f] = p0[f * PLANE + c];
        }
    }
    // after the planes of a step are staged: centres of plane k+1
    __device__ __forceinline__ void read_centres() {
#pragma unroll
        for (int f = 0; f < NF; ++f) cen[2][f] = s[2][f * PLANE + c];
    }
    // end of a step: k+1 becomes k, k becomes k-1
    __device__ __forceinline__ void shift() {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            cen[0][f] = cen[1][f];
            cen[1][f] = cen[2][f];
        }
    }
};

// offset s1 along axis a1 plus s2 along axis a2, as template arguments of at<>
#define OFF2(a1, s1, a2, s2)                                                            \
    ((a1) == 0 ? (s1) : 0) + ((a2) == 0 ? (s2) : 0),                                   \
        ((a1) == 1 ? (s1) : 0) + ((a2) == 1 ? (s2) : 0),                               \
        ((a1) == 2 ? (s1) : 0) + ((a2) == 2 ? (s2) : 0)
#define AT2(X, f, a1, s1, a2, s2) X.template at<OFF2(a1, s1, a2, s2)>(f)
#define AT1(X, f, a1, s1) AT2(X, f, a1, s1, a1, 0)

// Grid coefficients are read-only during a kernel: reading them through the
// constant address space marks the loads invariant, so uniform ones (the z
// set of a k-march step) become scalar loads and loop-invariant ones are
// hoisted -- none of them then waits behind the plane prefetch on the vector
// memory counter.
__device__ __forceinline__ double gc(const double *p, int i) {
    return ((const __attribute__((address_space(4))) double *)p)[i];
}

// Grid coefficients of one axis at one index i of that axis:
// 1/h[i], 1/h[i+1], 1/d[i], 1/d[i-1], w[i], w[i-1].  For x and y they are
// constant along a thread's k-march and live in registers; the z set is
// uniform across the block and reloaded per plane.
struct AxC {
    double ih0, ih1, id0, idm, w0, wm;
};

__device__ __forceinline__ AxC axc(const AxisDev &a, int i) {
    return AxC{gc(a.ih, i), gc(a.ih, i + 1), gc(a.id, i), gc(a.id, i - 1), gc(a.w, i),
               gc(a.w, i - 1)};
}

// field indices in the accessor: perturbation u v w T = 0..3, base = 4..7
// TERMS: the coupling terms carry the factors of fvk_set_terms (Coefs::f*);
// without it the expressions are those of the full operator.
template <int A, int Bt, bool TERMS, class Acc>
__device__ __forceinline__ void jrow_tangential(const AxC *C, const Acc &X, double wa,
                                                const Coefs &c, double &adv, double &lap) {
    const AxC &cB = C[Bt];
    const double wbp = cB.w0, wbm = cB.wm;
    // transporting component Bt at the edges (A-face, Bt-face jb and jb-1)
    const double Utp = (1.0 - wa) * AT1(X, 4 + Bt, A, 0) + wa * AT1(X, 4 + Bt, A, 1);
    const double Utm = (1.0 - wa) * AT1(X, 4 + Bt, Bt, -1) + wa * AT2(X, 4 + Bt, A, 1, Bt, -1);
    const double xtp = (1.0 - wa) * AT1(X, Bt, A, 0) + wa * AT1(X, Bt, A, 1);
    const double xtm = (1.0 - wa) * AT1(X, Bt, Bt, -1) + wa * AT2(X, Bt, A, 1, Bt, -1);
    // transported component A at the same edges
    const double xc = AT1(X, A, A, 0), Uc = AT1(X, 4 + A, A, 0);
    const double xpB = AT1(X, A, Bt, 1), xmB = AT1(X, A, Bt, -1);
    const double UpB = AT1(X, 4 + A, Bt, 1), UmB = AT1(X, 4 + A, Bt, -1);
    const double Uap = (1.0 - wbp) * Uc + wbp * UpB, Uam = (1.0 - wbm) * UmB + wbm * Uc;
    const double xap = (1.0 - wbp) * xc + wbp * xpB, xam = (1.0 - wbm) * xmB + wbm * xc;
    if (TERMS)
        adv += (c.fuv * (Utp * xap - Utm * xam) + c.fvu * (xtp * Uap - xtm * Uam)) * cB.ih0;
    else
        adv += (Utp * xap + xtp * Uap - Utm * xam - xtm * Uam) * cB.ih0;
    lap += ((xpB - xc) * cB.id0 - (xc - xmB) * cB.idm) * cB.ih0;
}

// nu Lap x_A - N_A(U, x_A) - N_A(x, U_A) (+ b T_f for A = z) at an interior A-face
template <int A, bool TERMS, class Acc>
__device__ __forceinline__ double jrow_mom(const AxC *C, const Acc &X, const Coefs &c) {
    const AxC &cA = C[A];
    const double xc = AT1(X, A, A, 0), xp = AT1(X, A, A, 1), xm = AT1(X, A, A, -1);
    const double Uc = AT1(X, 4 + A, A, 0), Up = AT1(X, 4 + A, A, 1), Um = AT1(X, 4 + A, A, -1);
    const double Ubp = 0.5 * (Uc + Up), Ubm = 0.5 * (Um + Uc);
    const double xbp = 0.5 * (xc + xp), xbm = 0.5 * (xm + xc);
    double adv = TERMS ? (c.fuv * (Ubp * xbp - Ubm * xbm) + c.fvu * (xbp * Ubp - xbm * Ubm)) * cA.id0
                       : (Ubp * xbp - Ubm * xbm + xbp * Ubp - xbm * Ubm) * cA.id0;
    double lap = ((xp - xc) * cA.ih1 - (xc - xm) * cA.ih0) * cA.id0;
    const double wa = cA.w0;
    jrow_tangential<A, (A + 1) % 3, TERMS>(C, X, wa, c, adv, lap);
    jrow_tangential<A, (A + 2) % 3, TERMS>(C, X, wa, c, adv, lap);
    double r = c.nu * lap - adv;
    const double bf = TERMS ? c.b * c.fb : c.b;
    if (A == 2) r += bf * ((1.0 - wa) * AT1(X, 3, 2, 0) + wa * AT1(X, 3, 2, 1));
    return r;
}

template <int A, bool TERMS, class Acc>
__device__ __forceinline__ void jrow_energy_axis(const AxC *C, const Acc &X, const Coefs &c,
                                                 double &adv, double &lap) {
    const AxC &cA = C[A];
    const double wp = cA.w0, wm = cA.wm, ih = cA.ih0;
    const double Tc = AT1(X, 3, A, 0), Tp = AT1(X, 3, A, 1), Tm = AT1(X, 3, A, -1);
    const double Hc = AT1(X, 7, A, 0), Hp = AT1(X, 7, A, 1), Hm = AT1(X, 7, A, -1);
    const double Tfp = (1.0 - wp) * Tc + wp * Tp, Tfm = (1.0 - wm) * Tm + wm * Tc;
    const double Hfp = (1.0 - wp) * Hc + wp * Hp, Hfm = (1.0 - wm) * Hm + wm * Hc;
    if (TERMS)
        adv += (c.fut[A] * (AT1(X, 4 + A, A, 0) * Tfp - AT1(X, 4 + A, A, -1) * Tfm) +
                c.fvt[A] * (AT1(X, A, A, 0) * Hfp - AT1(X, A, A, -1) * Hfm)) * ih;
    else
        adv += (AT1(X, 4 + A, A, 0) * Tfp - AT1(X, 4 + A, A, -1) * Tfm + AT1(X, A, A, 0) * Hfp -
                AT1(X, A, A, -1) * Hfm) * ih;
    lap += ((Tp - Tc) * cA.id0 - (Tc - Tm) * cA.idm) * ih;
}

template <bool TERMS, class Acc>
__device__ __forceinline__ double jrow_energy(const AxC *C, const Acc &X, const Coefs &c) {
    double adv = 0.0, lap = 0.0;
    jrow_energy_axis<0, TERMS>(C, X, c, adv, lap);
    jrow_energy_axis<1, TERMS>(C, X, c, adv, lap);
    jrow_energy_axis<2, TERMS>(C, X, c, adv, lap);
    return c.kappa * lap - adv;
}

// LDS-only workgroup barrier: orders LDS traffic without waiting for the
// global loads (prefetch) and stores (outputs) in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}


// Plane-relative addressing for the k-march through buffer resources: the
// descriptor of plane kk of a field (base, size in bytes) is block-uniform and
// lives in scalar registers, and a thread's in-plane byte offsets are fixed
// along the march (a plane is at most 1026^2 entries, well inside 32 bits), so
// no load or store needs per-access 64-bit address arithmetic.  A read at an
// offset past the descriptor's size returns 0 (buffer range checking): the
// halo entries outside the stored box are given such an offset, so they arrive
// already zeroed and the staging needs no mask.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr unsigned kOutside = 0x80000000u;   // beyond any plane: reads as 0
// s_waitcnt immediate (gfx9 encoding): vmcnt 0, expcnt and lgkmcnt not waited on
constexpr int kVmcntZero = 0x0F70;

__device__ __forceinline__ Rsrc plane_rsrc(const double *field, long plane_off, int bytes) {
    // dword 3 of a raw (untyped, stride 0) buffer descriptor on gfx9-family parts
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(field + plane_off), short(0),
                                             bytes, 0x00020000);
}
__device__ __forceinline__ double bload(Rsrc r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(off), 0, 0));
}
__device__ __forceinline__ void bstore(Rsrc r, unsigned off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, int(off), 0, 0);
}

// in-plane byte offsets of the thread's staged entries (kOutside outside the box)
template <class Tl>
struct PlaneSlots {
    unsigned off[Tl::PER];
};

template <class Tl>
__device__ __forceinline__ PlaneSlots<Tl> plane_slots(const Geo &g, int i0, int j0, int tid) {
    PlaneSlots<Tl> P;
#pragma unroll
    for (int q = 0; q < Tl::PER; ++q) {
        const int r = min(tid + q * Tl::NT, Tl::PLANE - 1);
        const int gi = i0 + r % TWP, gj = j0 + r / TWP;
        const bool ok = gi < g.np[0] && gj < g.np[1];
        P.off[q] = ok ? unsigned(gj * int(g.s[1]) + gi) * 8u : kOutside;
    }
    return P;
}

// global -> registers for one plane (tile + halo) of all fields.  Use-free:
// the NF * PER loads stay in flight across the whole step and are consumed
// only by put_plane_rel, one step later.  Slots past the plane are skipped.
template <class Tl>
__device__ __forceinline__ void fetch_plane_rel(const Geo &g, const double *const *fp,
                                                const PlaneSlots<Tl> &P, int kk, int tid,
                                                double (&reg)[NF][Tl::PER]) {
    const long base = long(kk) * g.s[2];
    const int bytes = int(g.s[2]) * 8;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const Rsrc r = plane_rsrc(fp[f], base, bytes);
#pragma unroll
        for (int q = 0; q < Tl::PER; ++q)
            if (q == 0 || tid + q * Tl::NT < Tl::PLANE) reg[f][q] = bload(r, P.off[q]);
    }
}

template <class Tl>
__device__ __forceinline__ void put_plane_rel(double *dst, int tid,
                                              const double (&reg)[NF][Tl::PER]) {
#pragma unroll
    for (int q = 0; q < Tl::PER; ++q) {
        const int r = tid + q * Tl::NT;
        if (r < Tl::PLANE) {
#pragma unroll
            for (int f = 0; f < NF; ++f) dst[f * Tl::PLANE + r] = reg[f][q];
        }
    }
}

__device__ __forceinline__ void store4(const Geo &g, double *yv, double *yT, int i, int j, int k,
                                       double u, double v, double w, double t) {
    const long p = pos(g, i, j, k);
    yv[p] = u;
    yv[p + g.F] = v;
    yv[p + 2 * g.F] = w;
    yT[p] = t;
}

// zero the wall neighbours of interior point (i, j) in plane kk (the stored
// entries outside the interior tile rows that this thread owns)
__device__ __forceinline__ void wall_writes(const Geo &g, double *yv, double *yT, int i, int j,
                                            int kk, double t_aa_lo, double t_aa_hi) {
    const int nx = g.n[0], ny = g.n[1];
    const int dis[3] = {0, i == 1 ? -1 : 0, i == nx ? 1 : 0};
    const int djs[3] = {0, j == 1 ? -1 : 0, j == ny ? 1 : 0};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if ((a == 0 && b == 0) || (a > 0 && dis[a] == 0) || (b > 0 && djs[b] == 0)) continue;
            const int di = dis[a], dj = djs[b];
            double t = 0.0;
            if (di == 0 && dj == -1) t = t_aa_lo;
            if (di == 0 && dj == 1) t = t_aa_hi;
            store4(g, yv, yT, i + di, j + dj, kk, 0.0, 0.0, 0.0, t);
        }
}

// wall_writes for plane k through the plane's four output descriptors
// (u v w T); `own` is the in-plane byte offset of (i, j)
__device__ __forceinline__ void wall_writes_rel(const Geo &g, const Rsrc *r4, unsigned own, int i,
                                                int j, double t_aa_lo, double t_aa_hi) {
    const int nx = g.n[0], ny = g.n[1];
    const int dis[3] = {0, i == 1 ? -1 : 0, i == nx ? 1 : 0};
    const int djs[3] = {0, j == 1 ? -1 : 0, j == ny ? 1 : 0};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if ((a == 0 && b == 0) || (a > 0 && dis[a] == 0) || (b > 0 && djs[b] == 0)) continue;
            const int di = dis[a], dj = djs[b];
            double t = 0.0;
            if (di == 0 && dj == -1) t = t_aa_lo;
            if (di == 0 && dj == 1) t = t_aa_hi;
            const unsigned o = own + unsigned((dj * int(g.s[1]) + di) * 8);
            bstore(r4[0], o, 0.0);
            bstore(r4[1], o, 0.0);
            bstore(r4[2], o, 0.0);
            bstore(r4[3], o, t);
        }
}

template <bool TERMS, int H>
__global__ __launch_bounds__(TX *H, 8 / H) void k_jac_tiled(Geo g, Coefs c, int span_aa,
                                                         const double *__restrict__ base,
                                                         const double *__restrict__ x,
                                                         double *__restrict__ yv,
                                                         double *__restrict__ yT, int kchunk) {
    using Tl = Tile<H>;
    __shared__ double lds[3][NF * Tl::PLANE];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    // XCD-aware tile order: hardware block b runs on XCD b % 8; give each XCD a
    // contiguous range of logical tiles
    const int nbx = gridDim.x, nby = gridDim.y, nbz = gridDim.z;
    const int nb = nbx * nby * nbz;
    const int b = (blockIdx.z * nby + blockIdx.y) * nbx + blockIdx.x;
    const int lb = int(xcd_remap(b, nb));
    const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
    const int i0 = bx * TX, j0 = by * H;           // halo origin (interior starts at +1)
    const int i = i0 + 1 + tx, j = j0 + 1 + ty;
    const int kb = 1 + bz * kchunk;
    const int ke = min(g.n[2], kb + kchunk - 1);
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const bool act = i <= nx && j <= ny;
    const long F = g.F;
    const double *fp[NF] = {x, x + F, x + 2 * F, x + 3 * F, base, base + F, base + 2 * F,
                            base + 3 * F};
    AxC C[3];
    C[0] = axc(g.ax[0], min(i, nx));
    C[1] = axc(g.ax[1], min(j, ny));
    const PlaneSlots<Tl> P = plane_slots<Tl>(g, i0, j0, tid);
    // this thread's output point within a plane (bytes; unused when !act)
    const unsigned own = unsigned(min(j, ny) * int(g.s[1]) + min(i, nx)) * 8u;
    const int pbytes = int(g.s[2]) * 8;
    double reg[NF][Tl::PER];
    fetch_plane_rel(g, fp, P, kb - 1, tid, reg);
    put_plane_rel<Tl>(lds[(kb - 1) % 3], tid, reg);
    fetch_plane_rel(g, fp, P, kb, tid, reg);
    put_plane_rel<Tl>(lds[kb % 3], tid, reg);
    // every load so far has been consumed; saying so here keeps the compiler's
    // wait analysis from carrying a stale pending load (a slot skipped on some
    // lanes) into the k-loop, where its wait would also drain the prefetch
    __builtin_amdgcn_s_waitcnt(kVmcntZero);
    fetch_plane_rel(g, fp, P, kb + 1, tid, reg);
    TileAcc<Tl::PLANE> X;
    X.c = (ty + 1) * TWP + tx + 1;
    lds_barrier();
    if (act) X.first_centres(lds[(kb - 1) % 3], lds[kb % 3]);
    for (int k = kb; k <= ke; ++k) {
        put_plane_rel<Tl>(lds[(k + 1) % 3], tid, reg);
        lds_barrier();
        // always issued (clamped to the last stored plane) so that the count
        // of loads in flight after this point is the same on every step
        fetch_plane_rel(g, fp, P, min(k + 2, nz + 1), tid, reg);
        C[2] = axc(g.ax[2], k);
        if (act) {
            X.s[0] = lds[(k - 1) % 3];
            X.s[1] = lds[k % 3];
            X.s[2] = lds[(k + 1) % 3];
            X.read_centres();
            // rows of (J + sigma I) x (sigma = 0 outside the shifted Krylov
            // operator); the centre values are already in registers
            const double u = (i <= nx - 1) ? jrow_mom<0, TERMS>(C, X, c) + c.sigma * X.cen[1][0]
                                           : 0.0;
            const double v = (j <= ny - 1) ? jrow_mom<1, TERMS>(C, X, c) + c.sigma * X.cen[1][1]
                                           : 0.0;
            const double w = (k <= nz - 1) ? jrow_mom<2, TERMS>(C, X, c) + c.sigma * X.cen[1][2]
                                           : 0.0;
            const double t = jrow_energy<TERMS>(C, X, c) + c.sigma * X.cen[1][3];
            const long pk = long(k) * g.s[2];
            const Rsrc r4[4] = {plane_rsrc(yv, pk, pbytes), plane_rsrc(yv + F, pk, pbytes),
                                plane_rsrc(yv + 2 * F, pk, pbytes), plane_rsrc(yT, pk, pbytes)};
            bstore(r4[0], own, u);
            bstore(r4[1], own, v);
            bstore(r4[2], own, w);
            bstore(r4[3], own, t);
            wall_writes_rel(g, r4, own, i, j, span_aa ? t : 0.0, span_aa ? t : 0.0);
            X.shift();
        }
        lds_barrier();
    }
    if (act) {
        if (kb == 1) {
            store4(g, yv, yT, i, j, 0, 0.0, 0.0, 0.0, 0.0);
            wall_writes(g, yv, yT, i, j, 0, 0.0, 0.0);
        }
        if (ke == nz) {
            store4(g, yv, yT, i, j, nz + 1, 0.0, 0.0, 0.0, 0.0);
            wall_writes(g, yv, yT, i, j, nz + 1, 0.0, 0.0);
        }
    }
}

// ---------------------------------------------------------------- transpose

// Transposed rows, written once over an accessor X of eight staged fields:
// 0..2 the momentum rows of Y restricted to the interior A-faces, 3 the energy
// rows of Y restricted to the cells (folded: with the insulated-wall
// extension, the wall entries added to their neighbours -- the transpose of
// Ext_T), 4..6 the base velocity U, 7 the base temperature Theta (zero
// outside the stored box).  X.at<d>(f) is field f at offset d.

// Transposed momentum-variable output for component A at stored position
// (i, j, k): collects every row in which x_A at this position appears, using
// the flux-adjoint form g = (row differences of Y) of each flux.
// Coefficients of one axis around index m, as the transposed rows use them:
// 1/h and 1/d at m-1, m, m+1; w at m-1, m (the arrays are padded to cover
// m = 0 and m = n+1).  The x and y sets are fixed along a thread's k-march
// and live in registers; the z set is uniform per step (scalar loads).
struct AxT {
    double ihm, ih0, ihp, idm, id0, idp, wm, w0;
};

__device__ __forceinline__ AxT axt(const AxisDev &a, int m) {
    return AxT{gc(a.ih, m - 1), gc(a.ih, m), gc(a.ih, m + 1), gc(a.id, m - 1),
               gc(a.id, m),     gc(a.id, m + 1), gc(a.w, m - 1), gc(a.w, m)};
}

template <int A, bool TERMS, class Acc>
__device__ __forceinline__ double jt_vel(const AxT *T, const Coefs &c, const Acc &X) {
    // factors of the coupling terms (TERMS); the normal part of the momentum
    // advection is half (U.grad) v and half (v.grad) U
    const double fn = TERMS ? 0.5 * (c.fuv + c.fvu) : 1.0;
    const double f3 = TERMS ? c.fuv : 1.0, f4 = TERMS ? c.fvu : 1.0;
    const double f5 = TERMS ? c.fvt[A] : 1.0;
    const AxT &TA = T[A];
    const double yc = AT1(X, A, A, 0), ym = AT1(X, A, A, -1), yp = AT1(X, A, A, 1);
    // viscous, normal direction
    double lapT = -(TA.ihp + TA.ih0) * TA.id0 * yc + TA.ih0 * TA.idm * ym + TA.ihp * TA.idp * yp;
    // advection, normal direction: - [Ubar(cell m) gn(m) + Ubar(cell m+1) gn(m+1)]
    const double uc = AT1(X, 4 + A, A, 0), um = AT1(X, 4 + A, A, -1), up = AT1(X, 4 + A, A, 1);
    double advT = 0.5 * (um + uc) * (ym * TA.idm - yc * TA.id0) +
                  0.5 * (uc + up) * (yc * TA.id0 - yp * TA.idp);
    if (TERMS) advT *= fn;
    const double wa = TA.w0;
#define FVK_JT_TANGENTIAL(Bt)                                                                \
    {                                                                                        \
        const AxT &TB = T[Bt];                                                               \
        const double ymB = AT1(X, A, Bt, -1), ypB = AT1(X, A, Bt, 1);                        \
        lapT += -(TB.id0 + TB.idm) * TB.ih0 * yc + TB.idm * TB.ihm * ymB +                   \
                TB.id0 * TB.ihp * ypB;                                                       \
        /* U_Bt interpolated along A to this A-face, at Bt-faces m and m-1 */                \
        const double ut_p = (1.0 - wa) * AT1(X, 4 + Bt, A, 0) + wa * AT1(X, 4 + Bt, A, 1);   \
        const double ut_m =                                                                  \
            (1.0 - wa) * AT1(X, 4 + Bt, Bt, -1) + wa * AT2(X, 4 + Bt, A, 1, Bt, -1);         \
        /* (3) x_A transported in the A-rows along Bt */                                     \
        const double gt_p = yc * TB.ih0 - ypB * TB.ihp;                                      \
        const double gt_m = ymB * TB.ihm - yc * TB.ih0;                                      \
        advT += f3 * (ut_p * (1.0 - TB.w0) * gt_p + ut_m * TB.wm * gt_m);                    \
        /* (4) x_A transporting U_Bt in the Bt-rows along A */                               \
        const double ybc = AT1(X, Bt, A, 0), ybA = AT1(X, Bt, A, 1);                         \
        const double ybm = AT1(X, Bt, Bt, -1), ybmA = AT2(X, Bt, A, 1, Bt, -1);              \
        const double gq_p = ybc * TA.ih0 - ybA * TA.ihp;                                     \
        const double gq_m = ybm * TA.ih0 - ybmA * TA.ihp;                                    \
        advT += f4 * ((1.0 - TB.w0) * ut_p * gq_p + TB.wm * ut_m * gq_m);                    \
    }
    FVK_JT_TANGENTIAL((A + 1) % 3)
    FVK_JT_TANGENTIAL((A + 2) % 3)
#undef FVK_JT_TANGENTIAL
    // (5) x_A transporting Theta in the energy rows
    const double thf = (1.0 - wa) * AT1(X, 7, A, 0) + wa * AT1(X, 7, A, 1);
    const double tc = AT1(X, 3, A, 0), tp = AT1(X, 3, A, 1);
    advT += f5 * (thf * (tc * TA.ih0 - tp * TA.ihp));
    return c.nu * lapT - advT;
}

template <int A, bool TERMS, class Acc>
__device__ __forceinline__ void jt_temp_axis(const AxT &TA, const Acc &X, const Coefs &c, double tc,
                                             double &lapT, double &advT) {
    const double tm = AT1(X, 3, A, -1), tp = AT1(X, 3, A, 1);
    lapT += -(TA.id0 + TA.idm) * TA.ih0 * tc + TA.idm * TA.ihm * tm + TA.id0 * TA.ihp * tp;
    const double uq = AT1(X, 4 + A, A, 0), uqm = AT1(X, 4 + A, A, -1);
    const double g_p = tc * TA.ih0 - tp * TA.ihp;
    const double g_m = tm * TA.ihm - tc * TA.ih0;
    if (TERMS)
        advT += c.fut[A] * (uq * (1.0 - TA.w0) * g_p + uqm * TA.wm * g_m);
    else
        advT += uq * (1.0 - TA.w0) * g_p + uqm * TA.wm * g_m;
}

template <bool TERMS, class Acc>
__device__ __forceinline__ double jt_temp(const AxT *T, const Coefs &c, const Acc &X) {
    const double tc = AT1(X, 3, 0, 0);
    double lapT = 0.0, advT = 0.0;
    jt_temp_axis<0, TERMS>(T[0], X, c, tc, lapT, advT);
    jt_temp_axis<1, TERMS>(T[1], X, c, tc, lapT, advT);
    jt_temp_axis<2, TERMS>(T[2], X, c, tc, lapT, advT);
    // buoyancy: the w-rows read T at the z-centres k and k+1
    const double buo = (1.0 - T[2].w0) * AT1(X, 2, 2, 0) + T[2].wm * AT1(X, 2, 2, -1);
    return c.kappa * lapT - advT + (TERMS ? c.b * c.fb : c.b) * buo;
}

// Tiled transposed Jacobian: the same k-march and LDS plane ring as
// k_jac_tiled, over ALL stored points (outputs live on walls too).  Plane
// entries are staged already masked (momentum rows on interior faces, energy
// rows on cells, folded) so the rows read them without tests.  The halo
// origin is one point below the tile in x and y; planes -1 and nz+2 are zero.
template <bool TERMS, int H>
__global__ __launch_bounds__(TX *H, 8 / H) void k_jacT_tiled(Geo g, Coefs c, int fold,
                                                          const double *__restrict__ base,
                                                          const double *__restrict__ yvel,
                                                          const double *__restrict__ yT,
                                                          double *__restrict__ x, int kchunk) {
    using Tl = Tile<H>;
    constexpr int PLANE = Tl::PLANE, NT_T = Tl::NT, PER_T = Tl::PER;
    __shared__ double lds[3][NF * PLANE];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const Blk B = xcd_block();
    const int i0 = B.x * TX - 1, j0 = B.y * H - 1;    // halo origin
    const int i = i0 + 1 + tx, j = j0 + 1 + ty;
    const int np2 = g.np[2];
    const int kb = B.z * kchunk;
    const int ke = min(np2 - 1, kb + kchunk - 1);
    const bool act = i < g.np[0] && j < g.np[1];
    const long F = g.F;
    double raw[NF][PER_T], fm[PER_T], fp[PER_T];
    // loads of plane kk (clamped addresses; masks applied in stage)
    auto fetch = [&](int kk) {
        const int kc = min(max(kk, 0), np2 - 1);
#pragma unroll
        for (int q = 0; q < PER_T; ++q) {
            if (q > 0 && tid + q * NT_T >= PLANE) continue;
            const int r = min(tid + q * NT_T, PLANE - 1);
            const int gi = min(max(i0 + r % TWP, 0), g.np[0] - 1);
            const int gj = min(max(j0 + r / TWP, 0), g.np[1] - 1);
            const long off = pos(g, gi, gj, kc);
#pragma unroll
            for (int f = 0; f < 3; ++f) raw[f][q] = yvel[f * F + off];
            raw[3][q] = yT[off];
#pragma unroll
            for (int f = 4; f < NF; ++f) raw[f][q] = base[(f - 4) * F + off];
            // neighbours for the fold (used on the two rows next to the
            // insulated walls; elsewhere a harmless reload of the same entry,
            // which keeps the loads unconditional)
            fm[q] = yT[off - (gj == 1 ? g.s[1] : 0)];
            fp[q] = yT[off + (gj == g.n[1] ? g.s[1] : 0)];
        }
    };
    auto stage = [&](int kk, double *dst) {
#pragma unroll
        for (int q = 0; q < PER_T; ++q) {
            const int r = tid + q * NT_T;
            if (r >= PLANE) continue;
            const int gi = i0 + r % TWP, gj = j0 + r / TWP;
            const bool box = gi >= 0 && gi < g.np[0] && gj >= 0 && gj < g.np[1] && kk >= 0 &&
                             kk < np2;
#pragma unroll
            for (int f = 0; f < 3; ++f)
                dst[f * PLANE + r] = face_row(g, f, gi, gj, kk) ? raw[f][q] : 0.0;
            double t = 0.0;
            if (cell_row(g, gi, gj, kk)) {
                t = raw[3][q];
                if (fold) {
                    if (gj == 1) t += fm[q];
                    if (gj == g.n[1]) t += fp[q];
                }
            }
            dst[3 * PLANE + r] = t;
#pragma unroll
            for (int f = 4; f < NF; ++f) dst[f * PLANE + r] = box ? raw[f][q] : 0.0;
        }
    };
    fetch(kb - 1);
    stage(kb - 1, lds[(kb + 2) % 3]);
    fetch(kb);
    stage(kb, lds[kb % 3]);
    fetch(kb + 1);
    TileAcc<PLANE> X;
    X.c = (ty + 1) * TWP + tx + 1;
    AxT T[3];
    T[0] = axt(g.ax[0], min(i, g.np[0] - 1));
    T[1] = axt(g.ax[1], min(j, g.np[1] - 1));
    lds_barrier();
    if (act) X.first_centres(lds[(kb + 2) % 3], lds[kb % 3]);
    for (int k = kb; k <= ke; ++k) {
        stage(k + 1, lds[(k + 1) % 3]);
        lds_barrier();
        fetch(k + 2);   // clamped inside: the same loads in flight on every step
        if (act) {
            X.s[0] = lds[(k + 2) % 3];
            X.s[1] = lds[k % 3];
            X.s[2] = lds[(k + 1) % 3];
            X.read_centres();
            T[2] = axt(g.ax[2], k);
            const long p = pos(g, i, j, k);
            // (J + sigma I)^T z with z the staged (masked, folded) input
            x[p] = jt_vel<0, TERMS>(T, c, X) + c.sigma * X.cen[1][0];
            x[p + F] = jt_vel<1, TERMS>(T, c, X) + c.sigma * X.cen[1][1];
            x[p + 2 * F] = jt_vel<2, TERMS>(T, c, X) + c.sigma * X.cen[1][2];
            x[p + 3 * F] = jt_temp<TERMS>(T, c, X) + c.sigma * X.cen[1][3];
            X.shift();
        }
        lds_barrier();
    }
}

// ---------------------------------------------------------------- SIMPLE pieces

__device__ __forceinline__ long cidx(const Geo &g, int i, int j, int k) {
    return (long(k - 1) * g.n[1] + (j - 1)) * g.n[0] + (i - 1);
}

// D v at interior cells (compact output).
// inverse face control volume 1/W of face A at (i, j, k): (1/d_A)(1/h_B)(1/h_C)
__device__ __forceinline__ double inv_w(const Geo &g, int A, int i, int j, int k) {
    const int idx[3] = {i, j, k};
    const int B = (A + 1) % 3, C = (A + 2) % 3;
    return g.ax[A].id[idx[A]] * g.ax[B].ih[idx[B]] * g.ax[C].ih[idx[C]];
}

// WIN: the divergence of W^-1 v (transposed projection), scaling on the fly
template <bool WIN>
__global__ __launch_bounds__(BX *BY) void k_div(Geo g, const double *__restrict__ v,
                                                double *__restrict__ dv) {
    const Blk B = xcd_block();
    const int i = B.x * BX + threadIdx.x + 1;
    const int j = B.y * BY + threadIdx.y + 1;
    const int k = B.z + 1;
    if (i > g.n[0] || j > g.n[1] || k > g.n[2]) return;
    const long p = pos(g, i, j, k);
    const int idx[3] = {i, j, k};
    double s = 0.0;
#pragma unroll
    for (int A = 0; A < 3; ++A) {
        double vp = v[A * g.F + p], vm = v[A * g.F + p - g.s[A]];
        if (WIN) {
            // wall faces are zero after the scaling (not interior faces)
            vp = idx[A] < g.n[A] ? vp * inv_w(g, A, i, j, k) : 0.0;
            vm = idx[A] > 1 ? vm * inv_w(g, A, A == 0 ? i - 1 : i, A == 1 ? j - 1 : j,
                                         A == 2 ? k - 1 : k)
                            : 0.0;
        }
        s += (vp - vm) * g.ax[A].ih[idx[A]];
    }
    dv[cidx(g, i, j, k)] = s;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    // wavefront reduction, then across the waves of the block
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    const int nw = (blockDim.x * blockDim.y + 63) / 64;
    double r = 0.0;
    if (t == 0) {
        for (int q = 0; q < nw; ++q) r = fmax(r, sh[q]);
    }
    return r;
}

// v_out = v_in - G phi on interior faces, p_out += phi, div_out = D v_out, and
// max |D v_out| over the grid.  Each thread owns the + faces of its cell; the
// x and y - faces are recomputed from v_in so the kernel is race-free
// (v_out != v_in).  A block owns a BX x BY column tile and kchunk consecutive
// planes, marching up in k: phi at k-1 and k and the corrected - face in z
// are carried in registers, so each phi and w value is read once.  Wall,
// edge and padding entries of v_out are written 0 (homogeneous no-slip,
// SIMPLE step 3) by the threads next to them, so v_out is fully defined.
// Block maxima of |D v_out| go to red[block]; a one-block kernel reduces them
// (per-block atomics on one address serialise in L2 and cost far more).
// WIN: v_in is read as W^-1 v_in (first pass of the transposed projection);
// WOUT: v_out is written as W v_out (its last pass); D v_out and its maximum
// are those of the unscaled result.
template <bool WIN, bool WOUT>
__global__ __launch_bounds__(BX *BY) void k_correct(Geo g, const double *__restrict__ vin,
                                                    const double *__restrict__ phi,
                                                    double *__restrict__ vout,
                                                    double *__restrict__ p_out,
                                                    double *__restrict__ div_out,
                                                    double *__restrict__ red, int kchunk) {
    __shared__ double sh[8];
    const Blk B = xcd_block();
    const int i = B.x * BX + threadIdx.x + 1;
    const int j = B.y * BY + threadIdx.y + 1;
    const int kb = 1 + B.z * kchunk;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int ke = min(nz, kb + kchunk - 1);
    double dmax = 0.0;
    if (i <= nx && j <= ny) {
        const long F = g.F, sxy = long(nx) * ny;
        const double *vu = vin, *vv = vin + F, *vw = vin + 2 * F;
        const double idxp = g.ax[0].id[i], idxm = g.ax[0].id[i - 1], ihx = g.ax[0].ih[i];
        const double idyp = g.ax[1].id[j], idym = g.ax[1].id[j - 1], ihy = g.ax[1].ih[j];
        // W^-1 factors of this column's faces (x and y faces: times 1/h_z(k))
        const double iwu = idxp * ihy, iwum = idxm * ihy, iwv = ihx * idyp, iwvm = ihx * idym,
                     iww = ihx * ihy;
        long c = cidx(g, i, j, kb);
        long p = pos(g, i, j, kb);
        double ph = phi[c];
        double wm = 0.0;   // corrected w on the - face of the current cell
        if (kb >= 2) {
            double w0 = vw[p - g.s[2]];
            if (WIN) w0 *= iww * g.ax[2].id[kb - 1];
            wm = w0 - (ph - phi[c - sxy]) * g.ax[2].id[kb - 1];
        }
        for (int k = kb; k <= ke; ++k) {
            const double ihzk = g.ax[2].ih[k];
            const double php = k < nz ? phi[c + sxy] : 0.0;
            double u0 = vu[p], u1 = vu[p - 1], v0 = vv[p], v1 = vv[p - g.s[1]], w0 = vw[p];
            if (WIN) {
                u0 *= iwu * ihzk;
                u1 *= iwum * ihzk;
                v0 *= iwv * ihzk;
                v1 *= iwvm * ihzk;
                w0 *= iww * g.ax[2].id[k];
            }
            const double up = i < nx ? u0 - (phi[c + 1] - ph) * idxp : 0.0;
            const double um = i >= 2 ? u1 - (ph - phi[c - 1]) * idxm : 0.0;
            const double vp = j < ny ? v0 - (phi[c + nx] - ph) * idyp : 0.0;
            const double vm = j >= 2 ? v1 - (ph - phi[c - nx]) * idym : 0.0;
            const double wp = k < nz ? w0 - (php - ph) * g.ax[2].id[k] : 0.0;
            if (WOUT) {
                vout[p] = up / (iwu * ihzk);
                vout[p + F] = vp / (iwv * ihzk);
                vout[p + 2 * F] = wp / (iww * g.ax[2].id[k]);
            } else {
                vout[p] = up;
                vout[p + F] = vp;
                vout[p + 2 * F] = wp;
            }
            const double dv = (up - um) * ihx + (vp - vm) * ihy + (wp - wm) * g.ax[2].ih[k];
            if (p_out) p_out[c] += ph;
            if (div_out) div_out[c] = dv;
            dmax = fmax(dmax, fabs(dv));
            // zero the velocity wall neighbours this cell owns (the stored
            // entries with an index 0 or n+1 next to it, edges and corners)
            const int lo[3] = {i == 1 ? -1 : 0, j == 1 ? -1 : 0, k == 1 ? -1 : 0};
            const int hi[3] = {i == nx ? 1 : 0, j == ny ? 1 : 0, k == nz ? 1 : 0};
            if (lo[0] | lo[1] | lo[2] | hi[0] | hi[1] | hi[2]) {
                for (int dk = lo[2]; dk <= hi[2]; ++dk)
                    for (int dj = lo[1]; dj <= hi[1]; ++dj)
                        for (int di = lo[0]; di <= hi[0]; ++di) {
                            if (di == 0 && dj == 0 && dk == 0) continue;
                            const long q = pos(g, i + di, j + dj, k + dk);
                            vout[q] = 0.0;
                            vout[q + F] = 0.0;
                            vout[q + 2 * F] = 0.0;
                        }
            }
            wm = wp;
            ph = php;
            c += sxy;
            p += g.s[2];
        }
    }
    const double r = block_max(dmax, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        red[B.lin] = r;
}

// zero-walls copy: dst = src on interior faces, 0 elsewhere (velocity fields)
__global__ void k_zero_vel_walls(Geo g, const double *__restrict__ src, double *__restrict__ dst) {
    const Blk B = xcd_block();
    const int i = B.x * BX + threadIdx.x;
    const int j = B.y * BY + threadIdx.y;
    const int k = B.z;
    if (i >= g.np[0] || j >= g.np[1] || k >= g.np[2]) return;
    const long p = pos(g, i, j, k);
#pragma unroll
    for (int A = 0; A < 3; ++A)
        dst[A * g.F + p] = face_row(g, A, i, j, k) ? src[A * g.F + p] : 0.0;
}

// Boundary-local temperature projection (eq. (21) for raw values whose
// insulated-wall nodes equal their neighbours): keep cells, Dirichlet wall
// nodes and edges <- 0, insulated y-wall nodes <- adjacent interior value.
__global__ void k_ext_T(Geo g, int span_aa, const double *__restrict__ src,
                        double *__restrict__ dst) {
    const Blk B = xcd_block();
    const int i = B.x * BX + threadIdx.x;
    const int j = B.y * BY + threadIdx.y;
    const int k = B.z;
    if (i >= g.np[0] || j >= g.np[1] || k >= g.np[2]) return;
    const long p = pos(g, i, j, k);
    double r = 0.0;
    if (cell_row(g, i, j, k)) {
        r = src[p];
    } else if (span_aa && i >= 1 && i <= g.n[0] && k >= 1 && k <= g.n[2]) {
        if (j == 0) r = src[p + g.s[1]];
        if (j == g.n[1] + 1) r = src[p - g.s[1]];
    }
    dst[p] = r;
}

// Face control-volume weights W = d_A h_B h_C of the interior A-faces.  The
// SIMPLE projection P is W-orthogonal (W G = -D^T V with V the cell volumes),
// so its Euclidean transpose is P^T = W P W^-1; this kernel applies W
// (inverse = 0) or W^-1 (inverse = 1) on interior faces and zeroes every other
// velocity entry.  In place is allowed.
__global__ void k_face_scale(Geo g, const double *__restrict__ src, double *__restrict__ dst,
                             int inverse) {
    const Blk B = xcd_block();
    const int i = B.x * BX + threadIdx.x;
    const int j = B.y * BY + threadIdx.y;
    const int k = B.z;
    if (i >= g.np[0] || j >= g.np[1] || k >= g.np[2]) return;
    const long p = pos(g, i, j, k);
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int A = 0; A < 3; ++A) {
        double r = 0.0;
        if (face_row(g, A, i, j, k)) {
            const int B = (A + 1) % 3, C = (A + 2) % 3;
            // 1/W = (1/d_A)(1/h_B)(1/h_C)
            const double iw = g.ax[A].id[idx[A]] * g.ax[B].ih[idx[B]] * g.ax[C].ih[idx[C]];
            r = inverse ? src[A * g.F + p] * iw : src[A * g.F + p] / iw;
        }
        dst[A * g.F + p] = r;
    }
}

// T part of P^T: transpose of the boundary-local extension.
__global__ void k_ext_T_T(Geo g, int span_aa, const double *__restrict__ src,
                          double *__restrict__ dst) {
    const Blk B = xcd_block();
    const int i = B.x * BX + threadIdx.x;
    const int j = B.y * BY + threadIdx.y;
    const int k = B.z;
    if (i >= g.np[0] || j >= g.np[1] || k >= g.np[2]) return;
    const long p = pos(g, i, j, k);
    double r = 0.0;
    if (cell_row(g, i, j, k)) {
        r = src[p];
        if (span_aa && j == 1) r += src[p - g.s[1]];
        if (span_aa && j == g.n[1]) r += src[p + g.s[1]];
    }
    dst[p] = r;
}

dim3 box_grid(const Geo &g) {
    return dim3((g.np[0] + BX - 1) / BX, (g.np[1] + BY - 1) / BY, g.np[2]);
}
dim3 cell_grid(const Geo &g) {
    return dim3((g.n[0] + BX - 1) / BX, (g.n[1] + BY - 1) / BY, g.n[2]);
}

}  // namespace

// column tiles x k-chunks of the correction kernel: >= ~1024 blocks, chunks
// of at least 4 planes where the grid allows
static dim3 correct_grid(const Geo &g, int *kchunk) {
    const int nbx = (g.n[0] + BX - 1) / BX, nby = (g.n[1] + BY - 1) / BY;
    int nchunk = (1024 + nbx * nby - 1) / (nbx * nby);
    nchunk = std::max(1, std::min(nchunk, std::max(1, g.n[2] / 4)));
    const int kc = (g.n[2] + nchunk - 1) / nchunk;
    if (kchunk) *kchunk = kc;
    return dim3(nbx, nby, (g.n[2] + kc - 1) / kc);
}

int correct_blocks(const Geo &g) {
    dim3 gr = correct_grid(g, nullptr);
    return int(gr.x * gr.y * gr.z);
}

// k-chunks per tile column.  The blocks run in rounds of 256 * per_cu
// resident blocks, and a block marching P planes costs about P + 2 plane
// steps (two planes staged before its first step); the chunk count minimises
// rounds x (P + 2), ties going to more blocks.  A count that leaves a last
// round nearly empty (e.g. 650 blocks on 512 slots) is what this avoids.
static int stencil_chunks(int tiles, int nk, int per_cu) {
    const long slots = 256L * per_cu;
    long best_cost = -1;
    int best = 1;
    for (int nc = 1; nc <= nk; ++nc) {
        const int planes = (nk + nc - 1) / nc;
        const int nc2 = (nk + planes - 1) / planes;   // chunks actually launched
        const long rounds = (long(tiles) * nc2 + slots - 1) / slots;
        const long cost = rounds * (planes + 2);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && nc2 > best)) {
            best_cost = cost;
            best = nc2;
        }
    }
    return best;
}

template <int H>
static void launch_jac_tiled(const Geo &g, Coefs c, int span_aa, const double *base,
                             const double *x, double *yv, double *yT, hipStream_t st) {
    // tiles of the interior plane; k split into chunks so the grid fills the
    // chip (8 / H resident blocks per CU) while each block keeps a long k-march
    const int nbx = (g.n[0] + TX - 1) / TX, nby = (g.n[1] + H - 1) / H;
    const int nchunk0 = stencil_chunks(nbx * nby, g.n[2], 8 / H);
    const int kchunk = (g.n[2] + nchunk0 - 1) / nchunk0;
    const int nchunk = (g.n[2] + kchunk - 1) / kchunk;
    const dim3 grid(nbx, nby, nchunk), block(TX, H);
    if (c.terms == FVK_TERMS_ALL)
        k_jac_tiled<false, H><<<grid, block, 0, st>>>(g, c, span_aa, base, x, yv, yT, kchunk);
    else
        k_jac_tiled<true, H><<<grid, block, 0, st>>>(g, c, span_aa, base, x, yv, yT, kchunk);
}

void launch_jacvec(const Geo &g, Coefs c, int span_aa, int ext, const double *base,
                   const double *x, double *yv, double *yT, hipStream_t st) {
    // 64 x 8 tiles (one 512-thread block per CU, 10 halo rows staged per 8
    // computed) once the grid is large enough to give every CU long marches;
    // 64 x 4 tiles (two blocks per CU, 6 rows per 4) below that
    const long cells = long(g.n[0]) * g.n[1] * g.n[2];
    if (cells >= 200L * 200 * 200)
        launch_jac_tiled<8>(g, c, span_aa && ext, base, x, yv, yT, st);
    else
        launch_jac_tiled<4>(g, c, span_aa && ext, base, x, yv, yT, st);
}

void launch_residual(const Geo &g, Coefs c, int span_aa, const double *base, double *F,
                     hipStream_t st) {
    (void)span_aa;
    k_jac<1><<<box_grid(g), dim3(BX, BY), 0, st>>>(g, c, 0, base, base, F, F + 3 * g.F);
}

template <int H>
static void launch_jacT_tiled(const Geo &g, Coefs c, int fold, const double *base,
                              const double *yvel, const double *yT, double *x, hipStream_t st) {
    // tiles of the whole stored plane; k (all np2 planes) split into chunks
    const int nbx = (g.np[0] + TX - 1) / TX, nby = (g.np[1] + H - 1) / H;
    const int nchunk0 = stencil_chunks(nbx * nby, g.np[2], 8 / H);
    const int kchunk = (g.np[2] + nchunk0 - 1) / nchunk0;
    const int nchunk = (g.np[2] + kchunk - 1) / kchunk;
    const dim3 grid(nbx, nby, nchunk), block(TX, H);
    if (c.terms == FVK_TERMS_ALL)
        k_jacT_tiled<false, H><<<grid, block, 0, st>>>(g, c, fold, base, yvel, yT, x, kchunk);
    else
        k_jacT_tiled<true, H><<<grid, block, 0, st>>>(g, c, fold, base, yvel, yT, x, kchunk);
}

void launch_jacvec_T(const Geo &g, Coefs c, int span_aa, int fold_ext, const double *base,
                     const double *yvel, const double *yT, double *x, hipStream_t st) {
    // tile heights as for the forward stencil
    const long cells = long(g.n[0]) * g.n[1] * g.n[2];
    if (cells >= 200L * 200 * 200)
        launch_jacT_tiled<8>(g, c, fold_ext && span_aa, base, yvel, yT, x, st);
    else
        launch_jacT_tiled<4>(g, c, fold_ext && span_aa, base, yvel, yT, x, st);
}

void launch_div(const Geo &g, const double *v, double *div, hipStream_t st, bool win) {
    if (win)
        k_div<true><<<cell_grid(g), dim3(BX, BY), 0, st>>>(g, v, div);
    else
        k_div<false><<<cell_grid(g), dim3(BX, BY), 0, st>>>(g, v, div);
}

void launch_correct_oop(const Geo &g, const double *vin, double *vout, const double *phi,
                        double *p_out, double *div_out, double *red, hipStream_t st, bool win,
                        bool wout) {
    int kchunk = 1;
    const dim3 gr = correct_grid(g, &kchunk);
    const dim3 bl(BX, BY);
    if (win && wout)
        k_correct<true, true><<<gr, bl, 0, st>>>(g, vin, phi, vout, p_out, div_out, red, kchunk);
    else if (win)
        k_correct<true, false><<<gr, bl, 0, st>>>(g, vin, phi, vout, p_out, div_out, red, kchunk);
    else if (wout)
        k_correct<false, true><<<gr, bl, 0, st>>>(g, vin, phi, vout, p_out, div_out, red, kchunk);
    else
        k_correct<false, false><<<gr, bl, 0, st>>>(g, vin, phi, vout, p_out, div_out, red, kchunk);
}

void launch_face_scale(const Geo &g, const double *src, double *dst, int inverse,
                       hipStream_t st) {
    k_face_scale<<<box_grid(g), dim3(BX, BY), 0, st>>>(g, src, dst, inverse);
}

void launch_ext_T(const Geo &g, int span_aa, const double *src, double *dst, hipStream_t st) {
    k_ext_T<<<box_grid(g), dim3(BX, BY), 0, st>>>(g, span_aa, src, dst);
}

void launch_ext_T_T(const Geo &g, int span_aa, const double *src, double *dst, hipStream_t st) {
    k_ext_T_T<<<box_grid(g), dim3(BX, BY), 0, st>>>(g, span_aa, src, dst);
}

void launch_zero_vel_walls(const Geo &g, const double *src, double *dst, hipStream_t st) {
    k_zero_vel_walls<<<box_grid(g), dim3(BX, BY), 0, st>>>(g, src, dst);
}

}  // namespace fvk
