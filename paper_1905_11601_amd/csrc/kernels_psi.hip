// Divergence-free projections of a velocity field onto the planes normal to
// one coordinate axis and their vector potentials: the visualisation of 3D
// flows by Psi_x, Psi_y, Psi_z used in the paper (Sec. 3.2).
//
// For the normal axis a with in-plane axes (b, c) in cyclic order, the
// projection keeps only the b- and c-components and removes their plane-wise
// gradient part (the 2D analogue of the SIMPLE step, W-orthogonal like it):
//   v' = Z v - G_bc L_bc^+ D_bc Z v,   L_bc = D_bc G_bc in every a-plane,
// Z: wall entries and the a-component set to 0.  Then v' = curl(psi e_a):
//   v'_b = d psi / d c,   v'_c = - d psi / d b,
// psi lives on the a-edges (b-faces x c-faces) and vanishes on the walls; it
// is the integral of h_c v'_b along c from the wall.
#include "fvk_internal.h"

namespace fvk {

namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ long pos3(const Geo &g, int i, int j, int k) {
    return (long(k) * g.np[1] + j) * g.np[0] + i;
}

// D_bc v at each interior cell (compact array), faces on the walls read as 0
__global__ __launch_bounds__(BX *BY) void k_div_plane(Geo g, const double *__restrict__ v,
                                                      double *__restrict__ div, int normal) {
    const int i = blockIdx.x * BX + threadIdx.x + 1;
    const int j = blockIdx.y * BY + threadIdx.y + 1;
    const int k = blockIdx.z + 1;
    if (i > g.n[0] || j > g.n[1] || k > g.n[2]) return;
    const int idx[3] = {i, j, k};
    const long p = pos3(g, i, j, k);
    double d = 0.0;
#pragma unroll
    for (int A = 0; A < 3; ++A) {
        if (A == normal) continue;
        const double *vA = v + A * g.F;
        const double up = idx[A] < g.n[A] ? vA[p] : 0.0;
        const double um = idx[A] > 1 ? vA[p - g.s[A]] : 0.0;
        d += (up - um) * g.ax[A].ih[idx[A]];
    }
    div[(long(k - 1) * g.n[1] + (j - 1)) * g.n[0] + (i - 1)] = d;
}

// in-plane components minus the plane-wise gradient at interior faces, every
// other entry 0; each thread reads only its own stored point of vin
__global__ __launch_bounds__(BX *BY) void k_correct_plane(Geo g, const double *vin,
                                                          const double *__restrict__ phi,
                                                          double *vout, int normal) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.np[0] || j >= g.np[1] || k >= g.np[2]) return;
    const int idx[3] = {i, j, k};
    const long p = pos3(g, i, j, k);
#pragma unroll
    for (int A = 0; A < 3; ++A) {
        bool row = A != normal;
#pragma unroll
        for (int B = 0; B < 3; ++B) {
            const int hi = (B == A) ? g.n[B] - 1 : g.n[B];
            if (idx[B] < 1 || idx[B] > hi) row = false;
        }
        double r = 0.0;
        if (row) {
            // cells idx and idx + e_A (1-based) on either side of the face
            const long c0 = (long(k - 1) * g.n[1] + (j - 1)) * g.n[0] + (i - 1);
            const long sc = A == 0 ? 1 : (A == 1 ? long(g.n[0]) : long(g.n[0]) * g.n[1]);
            r = vin[A * g.F + p] - (phi[c0 + sc] - phi[c0]) * g.ax[A].id[idx[A]];
        }
        vout[A * g.F + p] = r;
    }
}

// one thread per line (a-cell ia, b-face ib): psi = 0 at the c-wall, then
// psi(ic) = psi(ic - 1) + h_c(ic) v'_b(ic) over the c-cells; the stored entries
// outside (a index 0 or n_a + 1, b or c padding) are left as filled (0)
__global__ void k_psi_lines(Geo g, const double *__restrict__ vp, double *__restrict__ psi,
                            int a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
    const long nlines = long(g.n[a]) * (g.n[b] + 1);
    if (t >= nlines) return;
    const int ib = int(t % (g.n[b] + 1));
    const int ia = int(t / (g.n[b] + 1)) + 1;
    int idx[3];
    idx[a] = ia;
    idx[b] = ib;
    idx[c] = 0;
    const double *vb = vp + b * g.F;
    double acc = 0.0;
    psi[pos3(g, idx[0], idx[1], idx[2])] = 0.0;
    for (int ic = 1; ic <= g.n[c]; ++ic) {
        idx[c] = ic;
        const long p = pos3(g, idx[0], idx[1], idx[2]);
        acc += vb[p] / g.ax[c].ih[ic];
        psi[p] = acc;
    }
}

}  // namespace

void launch_div_plane(const Geo &g, const double *v, double *div, int normal, hipStream_t st) {
    const dim3 grid((g.n[0] + BX - 1) / BX, (g.n[1] + BY - 1) / BY, g.n[2]);
    k_div_plane<<<grid, dim3(BX, BY), 0, st>>>(g, v, div, normal);
}

void launch_correct_plane(const Geo &g, const double *vin, const double *phi, double *vout,
                          int normal, hipStream_t st) {
    const dim3 grid((g.np[0] + BX - 1) / BX, (g.np[1] + BY - 1) / BY, g.np[2]);
    k_correct_plane<<<grid, dim3(BX, BY), 0, st>>>(g, vin, phi, vout, normal);
}

void launch_psi_lines(const Geo &g, const double *vp, double *psi, int normal, hipStream_t st) {
    const int b = (normal + 1) % 3;
    launch_fill(psi, 0.0, size_t(g.F), st);
    const long nlines = long(g.n[normal]) * (g.n[b] + 1);
    const int nt = 256;
    k_psi_lines<<<unsigned((nlines + nt - 1) / nt), nt, 0, st>>>(g, vp, psi, normal);
}

}  // namespace fvk
