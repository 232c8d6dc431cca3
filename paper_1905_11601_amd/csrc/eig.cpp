// Host-side set-up: stretched staggered axes and the 1D eigendecompositions of
// the Neumann pressure-correction operator (paper Sec. 3.1, eqs (14)-(15)).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "fvk_internal.h"

namespace fvk {

static double face_map(double xi, int kind, double s) {
    switch (kind) {
        case FVK_GRID_SINE:  // eq. (22): x -> x - a sin(2 pi x)
            return xi - s * std::sin(2.0 * M_PI * xi);
        case FVK_GRID_TANH:
            return 0.5 * (1.0 + std::tanh(s * (2.0 * xi - 1.0)) / std::tanh(s));
        default:
            return xi;
    }
}

// Faces f[0..n] = map(i/n); centres at face midpoints plus the two wall nodes
// c[0] = 0, c[n+1] = 1; widths h[i] = f[i]-f[i-1]; spacings d[i] = c[i+1]-c[i];
// weights w[i] = (f[i]-c[i])/d[i] (w[0] = 0, w[n] = 1).
void build_axis(AxisHost &a, int n, int kind, double s) {
    a.n = n;
    a.f.assign(n + 1, 0.0);
    a.c.assign(n + 2, 0.0);
    a.h.assign(n + 2, 0.0);
    a.d.assign(n + 2, 0.0);
    a.w.assign(n + 2, 0.0);
    for (int i = 0; i <= n; ++i) a.f[i] = face_map(double(i) / n, kind, s);
    a.f[0] = 0.0;
    a.f[n] = 1.0;
    for (int i = 1; i <= n; ++i) a.c[i] = 0.5 * (a.f[i - 1] + a.f[i]);
    a.c[0] = 0.0;
    a.c[n + 1] = 1.0;
    for (int i = 1; i <= n; ++i) a.h[i] = a.f[i] - a.f[i - 1];
    for (int i = 0; i <= n; ++i) a.d[i] = a.c[i + 1] - a.c[i];
    // every grid kind is mirror-symmetric about 1/2; make the widths and
    // spacings exactly so (the subtractions above differ in the last bits
    // between mirrored pairs), so that the pressure operator D G is exactly
    // persymmetric and its eigenvectors split exactly into even and odd ones
    for (int i = 1; 2 * i <= n + 1; ++i) a.h[n + 1 - i] = a.h[i];
    for (int i = 0; 2 * i <= n; ++i) a.d[n - i] = a.d[i];
    for (int i = 0; i <= n; ++i) a.w[i] = (a.f[i] - a.c[i]) / a.d[i];
    a.w[0] = 0.0;
    a.w[n] = 1.0;
}

// Eigenvalues and orthonormal eigenvectors of the symmetric tridiagonal matrix
// with diagonal diag[0..n) and off-diagonal off[0..n-1) (off[i] couples i and
// i+1), by the implicit QL algorithm with Wilkinson-type shifts (Golub & Van
// Loan, Sec. 8.3).  Q is n x n row-major; column q is the eigenvector of
// lam[q].  Returns 0, or -1 if an eigenvalue needed more than 60 sweeps.
int tridiag_eig(int n, const double *diag, const double *off, double *lam, double *Q) {
    std::vector<double> d(diag, diag + n), e(n, 0.0);
    for (int i = 0; i + 1 < n; ++i) e[i] = off[i];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q[i * n + j] = (i == j) ? 1.0 : 0.0;
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < n; ++l) {
        int sweeps = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++sweeps > 60) return -1;
            // shift from the leading 2x2 block (eigenvalue closer to d[l])
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double sn = 1.0, cs = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                double f = sn * e[i], b = cs * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {  // exact split: undo the partial update
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * sn + 2.0 * cs * b;
                p = sn * r;
                d[i + 1] = g + p;
                g = cs * r - b;
                for (int k = 0; k < n; ++k) {  // accumulate the plane rotation
                    double qk1 = Q[k * n + i + 1], qk = Q[k * n + i];
                    Q[k * n + i + 1] = sn * qk + cs * qk1;
                    Q[k * n + i] = cs * qk - sn * qk1;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    for (int i = 0; i < n; ++i) lam[i] = d[i];
    return 0;
}

// D_aa = D_a G_a (Neumann): tridiagonal with V D_aa symmetric, V = diag(h).
// S = V^1/2 D_aa V^-1/2 = Q diag(lam) Q^T gives E = V^-1/2 Q, E^-1 = Q^T V^1/2.
// Eigenvalues sorted descending.  The null vector of S is known in closed
// form, q0 = V^1/2 1 / |V^1/2 1|; it replaces the computed one and the other
// eigenvectors are made orthogonal to it.  (Overwriting only column 0 of E and
// row 0 of E^-1 would leave E^-1 E - I of the size of the eigenvector error,
// ~ eps |S| / |lam_1|, which the three-dimensional solve then amplifies.)
void neumann_eig(const AxisHost &a, Eig1D &e) {
    const int n = a.n;
    std::vector<double> diag(n), off(std::max(n - 1, 1), 0.0);
    for (int i = 1; i <= n; ++i) {
        double dg = 0.0;
        if (i < n) dg -= 1.0 / (a.d[i] * a.h[i]);
        if (i > 1) dg -= 1.0 / (a.d[i - 1] * a.h[i]);
        diag[i - 1] = dg;
        if (i < n) off[i - 1] = 1.0 / (a.d[i] * std::sqrt(a.h[i] * a.h[i + 1]));
    }
    std::vector<double> lam(n), Q(size_t(n) * n);
    tridiag_eig(n, diag.data(), off.data(), lam.data(), Q.data());
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int p, int q) { return lam[p] > lam[q]; });
    std::vector<double> sh(n), q0(n), col(n);
    double len = 0.0;
    for (int i = 0; i < n; ++i) {
        sh[i] = std::sqrt(a.h[i + 1]);
        len += a.h[i + 1];
    }
    const double rl = 1.0 / std::sqrt(len);
    for (int i = 0; i < n; ++i) q0[i] = sh[i] * rl;
    e.n = n;
    e.lam.assign(n, 0.0);
    e.E.assign(size_t(n) * n, 0.0);
    e.Einv.assign(size_t(n) * n, 0.0);
    for (int q = 0; q < n; ++q) {
        const int src = order[q];
        e.lam[q] = q == 0 ? 0.0 : lam[src];
        if (q == 0) {
            col = q0;
        } else {
            for (int i = 0; i < n; ++i) col[i] = Q[size_t(i) * n + src];
            double dot = 0.0;
            for (int i = 0; i < n; ++i) dot += q0[i] * col[i];
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) {
                col[i] -= dot * q0[i];
                nrm += col[i] * col[i];
            }
            // fix the sign so the largest-magnitude component is positive
            double big = 0.0;
            for (int i = 0; i < n; ++i)
                if (std::fabs(col[i]) > std::fabs(big)) big = col[i];
            const double sc = (big < 0 ? -1.0 : 1.0) / std::sqrt(nrm);
            for (int i = 0; i < n; ++i) col[i] *= sc;
        }
        for (int i = 0; i < n; ++i) {
            e.E[size_t(i) * n + q] = col[i] / sh[i];
            e.Einv[size_t(q) * n + i] = col[i] * sh[i];
        }
    }
}

// Even/odd split of the same eigenbasis (exact for the mirror-symmetric
// axes): with N = 2m or 2m+1 cells, the eigenvectors of the persymmetric S
// are even or odd about the middle, and the two families are the
// eigenvectors of two tridiagonal matrices of order ne = N - m and no = m
// acting on the reduced coordinates c_i = sqrt(2) v_i (i < m; c_m = v_m for
// odd N).  An axis transform then becomes two half-size products:
//   forward  E^-1 x:  even coefficients = Ae (x_i + x_{N-1-i}),
//                     odd coefficients  = Ao (x_i - x_{N-1-i})
//                     (x_m itself in the last even column for odd N);
//   inverse  E y:     x_i = (Be y_e)_i + (Bo y_o)_i,
//                     x_{N-1-i} = (Be y_e)_i - (Bo y_o)_i, x_m = (Be y_e)_m.
// Coefficients are stored even modes first (each family descending in
// eigenvalue), so lam is permuted the same way; index 0 is the constant mode.
void neumann_eig_sym(const AxisHost &a, EigSym &e) {
    const int n = a.n, m = n / 2, ne = n - m, no = m;
    std::vector<double> diag(n), off(std::max(n - 1, 1), 0.0);
    for (int i = 1; i <= n; ++i) {
        double dg = 0.0;
        if (i < n) dg -= 1.0 / (a.d[i] * a.h[i]);
        if (i > 1) dg -= 1.0 / (a.d[i - 1] * a.h[i]);
        diag[i - 1] = dg;
        if (i < n) off[i - 1] = 1.0 / (a.d[i] * std::sqrt(a.h[i] * a.h[i + 1]));
    }
    // reduced tridiagonal matrices
    std::vector<double> de(ne), oe(std::max(ne - 1, 1), 0.0), dod(std::max(no, 1)),
        oo(std::max(no - 1, 1), 0.0);
    for (int i = 0; i < m; ++i) {
        de[i] = diag[i];
        dod[i] = diag[i];
    }
    for (int i = 0; i + 1 < m; ++i) {
        oe[i] = off[i];
        oo[i] = off[i];
    }
    if (n % 2 == 0) {
        de[m - 1] += off[m - 1];
        dod[m - 1] -= off[m - 1];
    } else {
        de[m] = diag[m];
        if (m > 0) oe[m - 1] = std::sqrt(2.0) * off[m - 1];
    }
    std::vector<double> sh(n);
    double len = 0.0;
    for (int i = 0; i < n; ++i) {
        sh[i] = std::sqrt(a.h[i + 1]);
        len += a.h[i + 1];
    }
    e.n = n;
    e.ne = ne;
    e.no = no;
    e.lam.assign(n, 0.0);
    e.A.assign(size_t(ne) * ne + size_t(no) * no, 0.0);
    e.B.assign(e.A.size(), 0.0);
    // reduced-coordinate weight: sqrt(2) off the middle, 1 at the middle
    auto red = [&](int i) { return (n % 2 == 1 && i == m) ? 1.0 : std::sqrt(2.0); };
    for (int fam = 0; fam < 2; ++fam) {
        const int k = fam == 0 ? ne : no;
        if (k == 0) continue;
        std::vector<double> lam(k), Q(size_t(k) * k);
        tridiag_eig(k, fam == 0 ? de.data() : dod.data(), fam == 0 ? oe.data() : oo.data(),
                    lam.data(), Q.data());
        std::vector<int> order(k);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int p, int q) { return lam[p] > lam[q]; });
        std::vector<double> c0(k), col(k);
        if (fam == 0) {   // closed-form null vector in reduced coordinates
            const double rl = 1.0 / std::sqrt(len);
            for (int i = 0; i < k; ++i) c0[i] = red(i) * sh[i] * rl;
        }
        double *Mf = e.A.data() + (fam == 0 ? 0 : size_t(ne) * ne);
        double *Mi = e.B.data() + (fam == 0 ? 0 : size_t(ne) * ne);
        for (int q = 0; q < k; ++q) {
            const int src = order[q];
            e.lam[(fam == 0 ? 0 : ne) + q] = (fam == 0 && q == 0) ? 0.0 : lam[src];
            if (fam == 0 && q == 0) {
                col = c0;
            } else {
                for (int i = 0; i < k; ++i) col[i] = Q[size_t(i) * k + src];
                double nrm = 0.0;
                if (fam == 0) {
                    double dot = 0.0;
                    for (int i = 0; i < k; ++i) dot += c0[i] * col[i];
                    for (int i = 0; i < k; ++i) col[i] -= dot * c0[i];
                }
                for (int i = 0; i < k; ++i) nrm += col[i] * col[i];
                double big = 0.0;
                for (int i = 0; i < k; ++i)
                    if (std::fabs(col[i]) > std::fabs(big)) big = col[i];
                const double sc = (big < 0 ? -1.0 : 1.0) / std::sqrt(nrm);
                for (int i = 0; i < k; ++i) col[i] *= sc;
            }
            // full eigenvector entries v_i = col_i / red(i); E^-1 rows carry
            // sqrt(h), E columns 1 / sqrt(h)
            for (int i = 0; i < k; ++i) {
                const double v = col[i] / red(i);
                Mf[size_t(q) * k + i] = v * sh[i];
                Mi[size_t(i) * k + q] = v / sh[i];
            }
        }
    }
}

}  // namespace fvk
