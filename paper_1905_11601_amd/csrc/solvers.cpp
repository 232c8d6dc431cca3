// Newton iteration for steady states (paper Sec. 3.1, Newton steps 1-4) with
// its linear solves: restarted GMRES(m) until converged or saturated, then
// BiCGstab(2) (Sleijpen & Fokkema 1993) started from the GMRES iterate, as the
// paper describes for grids of 150^3 and finer.  Every Krylov vector is a
// simple_krylov_vec call; orthogonalisation and vector updates run in the
// library's kernels; only the small Hessenberg / Givens / BiCGstab scalars
// live on the host.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fvk_internal.h"

using namespace fvk;

namespace {

// Convergence log to stderr when the environment variable FVK_VERBOSE is set
// (one line per Newton iteration, GMRES cycle and 100 BiCGstab(2) iterations).
bool verbose() {
    static const bool v = std::getenv("FVK_VERBOSE") != nullptr;
    return v;
}

struct Dev {
    fvk_ctx *ctx;
    size_t n;
    fvk_status st = FVK_OK;

    double dot(const double *x, const double *y) {
        if (st != FVK_OK) return 0.0;
        double out = 0.0;
        st = fvk_multidot(ctx, x, n, 1, y, n, &out);
        return out;
    }
    double nrm(const double *x) { return std::sqrt(dot(x, x)); }
    // y = a x + b y
    void axpby(double *y, double a, const double *x, double b) {
        launch_axpby(y, a, x, b, n, ctx->stream);
    }
    void copy(double *dst, const double *src) { launch_copy(dst, src, n, ctx->stream); }
    void fill(double *y, double v) { launch_fill(y, v, n, ctx->stream); }
    void apply(const double *base, const double *x, double *y) {
        if (st != FVK_OK) return;
        st = simple_krylov_vec(ctx, base, x, y, nullptr, 0, nullptr, nullptr);
    }
};

fvk_status dmalloc(fvk_ctx *ctx, double **p, size_t count) {
    if (hipMalloc(reinterpret_cast<void **>(p), count * sizeof(double)) != hipSuccess) {
        *p = nullptr;
        ctx->err = "newton_step: device allocation failed";
        return FVK_ENOMEM;
    }
    return FVK_OK;
}

double max_abs(Dev &d, const double *x) {
    fvk_ctx *ctx = d.ctx;
    const int nb = multidot_blocks(d.n);
    launch_absmax(x, d.n, ctx->ws.red, nb, ctx->stream);
    launch_max_reduce(ctx->ws.red, nb, ctx->ws.dev_scalars + 6, nullptr, nullptr, 0.0,
                      ctx->stream);
    double m = 0.0;
    if (hipMemcpyAsync(ctx->ws.host_pinned, ctx->ws.dev_scalars + 6, sizeof(double),
                       hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        d.st = FVK_EHIP;
        return 0.0;
    }
    m = ctx->ws.host_pinned[0];
    return m;
}

// GMRES(m) on A x = b from x (in/out).  Returns the final true relative
// residual in *rel; *cycles counts restarts; stops on convergence (rel < tol)
// or saturation (a cycle reducing |r| by less than sat_ratio).
fvk_status gmres(Dev &d, const double *base, const double *b, double *x, double *V, int m,
                 int max_cycles, double tol, double sat_ratio, double *rel, int *cycles,
                 int *nvec, double *r, double *tmp) {
    fvk_ctx *ctx = d.ctx;
    const size_t n = d.n;
    const double bn = d.nrm(b);
    if (d.st != FVK_OK) return d.st;
    if (bn == 0.0) {
        d.fill(x, 0.0);
        *rel = 0.0;
        return FVK_OK;
    }
    // r = b - A x
    d.apply(base, x, tmp);
    d.copy(r, b);
    d.axpby(r, -1.0, tmp, 1.0);
    double beta = d.nrm(r);
    if (d.st != FVK_OK) return d.st;
    std::vector<double> H(size_t(m + 1) * m), Ha(size_t(m + 1) * m), cs(m), sn(m), gvec(m + 1),
        hcol(m + 2), y(m);
    *cycles = 0;
    while (beta / bn > tol && *cycles < max_cycles) {
        d.copy(V, r);
        launch_scale(V, 1.0 / beta, n, ctx->stream);
        std::fill(gvec.begin(), gvec.end(), 0.0);
        std::fill(Ha.begin(), Ha.end(), 0.0);
        gvec[0] = beta;
        int jend = 0;
        // Column c of the Arnoldi matrix Ha is final once step c+1 (or the
        // closing arnoldi_finish) has re-orthogonalised v_{c+1}; the Givens
        // rotations and the residual estimate follow one step behind.
        auto column = [&](int c) {
            for (int i = 0; i <= c + 1; ++i) hcol[i] = Ha[size_t(i) * m + c];
            for (int i = 0; i < c; ++i) {   // previous rotations
                const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
                hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
                hcol[i] = t;
            }
            const double hh = std::hypot(hcol[c], hcol[c + 1]);
            cs[c] = hh > 0 ? hcol[c] / hh : 1.0;
            sn[c] = hh > 0 ? hcol[c + 1] / hh : 0.0;
            hcol[c] = hh;
            hcol[c + 1] = 0.0;
            gvec[c + 1] = -sn[c] * gvec[c];
            gvec[c] = cs[c] * gvec[c];
            for (int i = 0; i <= c; ++i) H[size_t(i) * m + c] = hcol[i];
            jend = c + 1;
            return std::fabs(gvec[c + 1]) / bn <= tol;
        };
        bool done = false;
        for (int j = 0; j < m && !done; ++j) {
            fvk_status s = arnoldi_step_lagged(ctx, base, V, n, j, Ha.data(), m, 0);
            if (s != FVK_OK && s != FVK_EBREAKDOWN) return s;
            ++*nvec;
            if (j > 0) done = column(j - 1) || s == FVK_EBREAKDOWN;
            else if (s == FVK_EBREAKDOWN) return s;   // the start vector vanished
        }
        if (!done) {
            const fvk_status s = arnoldi_finish(ctx, V, n, m, Ha.data(), m);
            if (s != FVK_OK && s != FVK_EBREAKDOWN) return s;
            column(m - 1);
        }
        for (int i = jend - 1; i >= 0; --i) {   // back substitution R y = g
            double sacc = gvec[i];
            for (int k = i + 1; k < jend; ++k) sacc -= H[size_t(i) * m + k] * y[k];
            y[i] = sacc / H[size_t(i) * m + i];
        }
        fvk_status s = fvk_multiaxpy(ctx, x, 1.0, V, n, jend, y.data(), n);
        if (s != FVK_OK) return s;
        ++*cycles;
        d.apply(base, x, tmp);
        d.copy(r, b);
        d.axpby(r, -1.0, tmp, 1.0);
        const double beta_new = d.nrm(r);
        if (d.st != FVK_OK) return d.st;
        const bool saturated = beta_new > sat_ratio * beta;
        if (verbose())
            std::fprintf(stderr, "[fvk] gmres cycle %d: %d vectors, |r|/|b| %.3e (estimate %.3e)%s\n",
                         *cycles, jend, beta_new / bn, std::fabs(gvec[jend]) / bn,
                         saturated ? " saturated" : "");
        beta = beta_new;
        if (saturated) break;
    }
    *rel = beta / bn;
    return FVK_OK;
}

// BiCGstab(2) on A x = b from x (in/out); work holds 8 vectors, keep two
// (the best iterate and the starting one).  Past its attainable accuracy
// BiCGstab can wander off and its recursively updated residual drifts from
// the true one: the best iterate seen is kept, the iteration stops once the
// residual exceeds 1e4 times the best one or the best has improved by less
// than 10% over 250 iterations, the recursive residual is replaced by the
// true one every 250 iterations, and the result is the starting x unless its
// true residual is smaller.
fvk_status bicgstab2(Dev &d, const double *base, const double *b, double *x, double *work,
                     double *keep, int max_it, double tol, double *rel, int *its, int *nvec) {
    double *xbest = keep, *xstart = keep + d.n;
    const size_t n = d.n;
    double *r0t = work, *r[3] = {work + n, work + 2 * n, work + 3 * n};
    double *u[3] = {work + 4 * n, work + 5 * n, work + 6 * n};
    double *tmp = work + 7 * n;
    const int L = 2;
    const double bn = d.nrm(b);
    if (d.st != FVK_OK) return d.st;
    if (bn == 0.0) {
        *rel = 0.0;
        return FVK_OK;
    }
    d.apply(base, x, tmp);
    ++*nvec;
    d.copy(r[0], b);
    d.axpby(r[0], -1.0, tmp, 1.0);
    d.copy(r0t, r[0]);
    d.fill(u[0], 0.0);
    double rho0 = 1.0, alpha = 0.0, omega = 1.0;
    double res = d.nrm(r[0]) / bn;
    const double res_start = res;
    double best = res, best_mark = res;
    d.copy(xbest, x);
    d.copy(xstart, x);
    *its = 0;
    // a breakdown of the BiCG recurrences (rho, gamma or omega zero or not
    // finite) restarts them from the true residual with a fresh shadow
    // residual; two breakdowns in a row end the iteration
    int breakdowns = 0;
    while (res > tol && *its < max_it && d.st == FVK_OK) {
        rho0 = -omega * rho0;
        bool broke = !(std::isfinite(rho0) && rho0 != 0.0);
        for (int j = 0; j < L && !broke; ++j) {
            const double rho1 = d.dot(r[j], r0t);
            const double beta = alpha * rho1 / rho0;
            rho0 = rho1;
            for (int i = 0; i <= j; ++i) d.axpby(u[i], 1.0, r[i], -beta);   // u_i = r_i - beta u_i
            d.apply(base, u[j], u[j + 1]);
            ++*nvec;
            const double gamma = d.dot(u[j + 1], r0t);
            if (!(std::isfinite(gamma) && gamma != 0.0 && std::isfinite(beta))) {
                broke = true;
                break;
            }
            alpha = rho0 / gamma;
            for (int i = 0; i <= j; ++i) d.axpby(r[i], -alpha, u[i + 1], 1.0);
            d.apply(base, r[j], r[j + 1]);
            ++*nvec;
            d.axpby(x, alpha, u[0], 1.0);
        }
        if (broke) {
            if (++breakdowns >= 2 || d.st != FVK_OK) break;
            if (verbose())
                std::fprintf(stderr, "[fvk] bicgstab(2) breakdown at it %d: restart\n", *its);
            if (best < res) d.copy(x, xbest);
            d.apply(base, x, tmp);
            ++*nvec;
            d.copy(r[0], b);
            d.axpby(r[0], -1.0, tmp, 1.0);
            d.copy(r0t, r[0]);
            d.fill(u[0], 0.0);
            rho0 = 1.0;
            alpha = 0.0;
            omega = 1.0;
            res = d.nrm(r[0]) / bn;
            continue;
        }
        breakdowns = 0;
        // minimal-residual part (modified Gram-Schmidt on r_1..r_L)
        double tau[L + 1][L + 1] = {}, sig[L + 1] = {}, gp[L + 1] = {}, g[L + 1] = {},
               g2[L + 1] = {};
        for (int j = 1; j <= L; ++j) {
            for (int i = 1; i < j; ++i) {
                tau[i][j] = d.dot(r[j], r[i]) / sig[i];
                d.axpby(r[j], -tau[i][j], r[i], 1.0);
            }
            sig[j] = d.dot(r[j], r[j]);
            if (sig[j] == 0.0) sig[j] = 1e-300;
            gp[j] = d.dot(r[0], r[j]) / sig[j];
        }
        g[L] = gp[L];
        omega = g[L];
        for (int j = L - 1; j >= 1; --j) {
            double sacc = gp[j];
            for (int i = j + 1; i <= L; ++i) sacc -= tau[j][i] * g[i];
            g[j] = sacc;
        }
        for (int j = 1; j <= L - 1; ++j) {
            double sacc = g[j + 1];
            for (int i = j + 1; i <= L - 1; ++i) sacc += tau[j][i] * g[i + 1];
            g2[j] = sacc;
        }
        d.axpby(x, g[1], r[0], 1.0);
        d.axpby(r[0], -gp[L], r[L], 1.0);
        d.axpby(u[0], -g[L], u[L], 1.0);
        for (int j = 1; j <= L - 1; ++j) {
            d.axpby(u[0], -g[j], u[j], 1.0);
            d.axpby(x, g2[j], r[j], 1.0);
            d.axpby(r[0], -gp[j], r[j], 1.0);
        }
        ++*its;
        res = d.nrm(r[0]) / bn;
        if (verbose() && (*its % 100 == 0 || res <= tol))
            std::fprintf(stderr, "[fvk] bicgstab(2) it %d: |r|/|b| %.3e\n", *its, res);
        if (res < best) {
            best = res;
            d.copy(xbest, x);
        } else if (!(res < 1e4 * best)) {
            break;
        }
        if (*its % 250 == 0) {
            if (best > 0.9 * best_mark) break;
            best_mark = best;
            // residual replacement: r_0 <- b - A x
            d.apply(base, x, tmp);
            ++*nvec;
            d.copy(r[0], b);
            d.axpby(r[0], -1.0, tmp, 1.0);
            res = d.nrm(r[0]) / bn;
        }
    }
    if (best < res) d.copy(x, xbest);
    // the true residual of the candidate decides against the start
    d.apply(base, x, tmp);
    ++*nvec;
    d.copy(r[0], b);
    d.axpby(r[0], -1.0, tmp, 1.0);
    const double res_true = d.nrm(r[0]) / bn;
    if (verbose())
        std::fprintf(stderr, "[fvk] bicgstab(2) done after %d its: true |r|/|b| %.3e (start %.3e)\n",
                     *its, res_true, res_start);
    if (!(res_true < res_start)) {
        d.copy(x, xstart);
        *rel = res_start;
    } else {
        *rel = res_true;
    }
    return d.st;
}

}  // namespace

extern "C" {

void fvk_newton_defaults(fvk_newton_opts *o) {
    if (!o) return;
    o->tol = 1e-10;
    o->gmres_m = 100;
    o->gmres_max_restarts = 50;
    o->sat_ratio = 0.9;
    o->bicgstab_max_it = 5000;
    o->lin_tol = 1e-8;
    o->max_newton = 12;
}

namespace {

// The linear solves of the Newton iteration are on A itself: the spectral
// shift of fvk_set_shift (an eigenvalue-solver setting) is switched off for
// the duration of a call and restored afterwards.
struct NoShift {
    fvk_ctx *ctx;
    double saved;
    explicit NoShift(fvk_ctx *c) : ctx(c), saved(c->shift) { c->shift = 0.0; }
    ~NoShift() { ctx->shift = saved; }
};

// GMRES(m) then BiCGstab(2) on A x = b; V: (m+1) vectors, work: 10 vectors.
fvk_status linear_solve(Dev &d, const double *base, const double *b, double *x, double *V,
                        double *work, const fvk_newton_opts &o, fvk_newton_report &R) {
    const size_t n = d.n;
    double rel = 1.0;
    int cyc = 0;
    fvk_status st = gmres(d, base, b, x, V, o.gmres_m, o.gmres_max_restarts, o.lin_tol,
                          o.sat_ratio, &rel, &cyc, &R.krylov_vecs, work, work + n);
    R.gmres_cycles += cyc;
    if (st != FVK_OK) return st;
    if (rel > o.lin_tol && o.bicgstab_max_it > 0) {
        int its = 0;
        st = bicgstab2(d, base, b, x, work + 2 * n, V, o.bicgstab_max_it, o.lin_tol, &rel, &its,
                       &R.krylov_vecs);
        R.bicgstab_its += its;
        if (st != FVK_OK) return st;
    }
    R.lin_rel_res = rel;
    R.lin_status = rel <= o.lin_tol ? FVK_OK : FVK_ENOCONV;
    return FVK_OK;
}

}  // namespace

fvk_status fvk_linear_solve(fvk_ctx *ctx, const double *base, const double *b, double *x,
                            const fvk_newton_opts *opts, fvk_newton_report *rep) {
    if (!ctx || !base || !b || !x) return FVK_EINVAL;
    fvk_newton_opts o;
    fvk_newton_defaults(&o);
    if (opts) o = *opts;
    if (o.gmres_m < 1 || o.gmres_m > 400) return FVK_EINVAL;
    const NoShift unshifted(ctx);
    fvk_newton_report R;
    std::memset(&R, 0, sizeof(R));
    size_t ntot = 0;
    fvk_layout(ctx, nullptr, nullptr, &ntot);
    Dev d{ctx, ntot};
    double *V = nullptr, *work = nullptr;
    fvk_status st = dmalloc(ctx, &V, size_t(o.gmres_m + 1) * ntot);
    if (st == FVK_OK) st = dmalloc(ctx, &work, 10 * ntot);
    if (st == FVK_OK) st = linear_solve(d, base, b, x, V, work, o, R);
    if (st == FVK_OK) {   // return the solution in S (see newton_step)
        st = fvk_project(ctx, x, work, 0);
        if (st == FVK_OK) d.copy(x, work);
    }
    if (st == FVK_OK && R.lin_status != FVK_OK) {
        st = FVK_ENOCONV;
        ctx->err = "fvk_linear_solve: tolerance not reached";
    }
    if (V) (void)hipFree(V);
    if (work) (void)hipFree(work);
    if (rep) *rep = R;
    return st;
}

fvk_status newton_step(fvk_ctx *ctx, double *base, const fvk_newton_opts *opts,
                       fvk_newton_report *rep) {
    if (!ctx || !base) return FVK_EINVAL;
    fvk_newton_opts o;
    fvk_newton_defaults(&o);
    if (opts) o = *opts;
    if (o.gmres_m < 1 || o.gmres_m > 400 || o.max_newton < 0) return FVK_EINVAL;
    const NoShift unshifted(ctx);
    fvk_newton_report R;
    std::memset(&R, 0, sizeof(R));
    size_t ntot = 0;
    fvk_layout(ctx, nullptr, nullptr, &ntot);
    Dev d{ctx, ntot};
    double *V = nullptr, *b = nullptr, *x = nullptr, *work = nullptr;
    fvk_status st = FVK_OK;
    if ((st = dmalloc(ctx, &V, size_t(o.gmres_m + 1) * ntot)) != FVK_OK) return st;
    if ((st = dmalloc(ctx, &b, ntot)) != FVK_OK) goto done;
    if ((st = dmalloc(ctx, &x, ntot)) != FVK_OK) goto done;
    if ((st = dmalloc(ctx, &work, 10 * ntot)) != FVK_OK) goto done;
    for (int it = 0; it <= o.max_newton; ++it) {
        st = fv_residual(ctx, base, b, 1);
        if (st != FVK_OK) goto done;
        const double res = max_abs(d, b);
        if (d.st != FVK_OK) {
            st = d.st;
            goto done;
        }
        if (it == 0) R.res_before = res;
        R.res_after = res;
        if (verbose()) std::fprintf(stderr, "[fvk] newton it %d: max|P F| %.3e\n", it, res);
        if (res < o.tol || it == o.max_newton) break;
        // no over-solving: a linear residual below 1% of the Newton tolerance
        // is enough, and iterating further only adds rounding noise
        const double bn2 = d.nrm(b);
        fvk_newton_opts ol = o;
        if (bn2 > 0.0) ol.lin_tol = std::fmax(o.lin_tol, 1e-2 * o.tol / bn2);
        d.fill(x, 0.0);
        st = linear_solve(d, base, b, x, V, work, ol, R);
        if (st != FVK_OK) goto done;
        // delta belongs to the constraint subspace S (divergence-free,
        // homogeneous boundary values).  Iterations run past their attainable
        // accuracy pick up gradient fields from the rounding of the Poisson
        // solves, amplified by large coefficients, and the rest of delta then
        // compensates for them in A delta; without this projection they would
        // accumulate in U, giving a state with P F = 0 but D U != 0.
        st = fvk_project(ctx, x, work, 0);
        if (st != FVK_OK) goto done;
        d.axpby(base, -1.0, work, 1.0);   // U <- U - delta
        ++R.newton_its;
    }
    if (R.res_after >= o.tol) {
        st = FVK_ENOCONV;
        ctx->err = "newton_step: residual above tolerance after max_newton iterations";
    }
done:
    if (V) (void)hipFree(V);
    if (b) (void)hipFree(b);
    if (x) (void)hipFree(x);
    if (work) (void)hipFree(work);
    if (rep) *rep = R;
    return st;
}

}  // extern "C"
