/*
 * fvk -- Krylov-vector engine for the linear-stability / Newton solver of
 * buoyancy convection in a laterally heated cube (Gelfgat, arXiv:1905.11601),
 * for AMD Instinct MI355X (gfx950).
 *
 * C ABI.  All `double *` arguments named base, x, y, F, V, p_out, w are DEVICE
 * pointers to caller-owned, contiguous FP64 buffers (e.g. torch tensors) in
 * the layout reported by fvk_layout(); `h_col`, `Q`, `out` and the grid-query
 * arrays are HOST pointers.  The context owns every workspace it needs
 * (allocated once in fvk_create, sized for the grid).  All work is enqueued
 * on the HIP stream given to fvk_create / fvk_set_stream; calls that return
 * host values synchronise that stream.  A context is not thread-safe; use one
 * per stream.  Errors are status codes with a message from fvk_last_error();
 * no call aborts or throws.
 *
 * Layout of a 4-field vector (Krylov vector, base flow, residual):
 *   field f in {0:u, 1:v, 2:w, 3:T} starts at f * field_len doubles;
 *   each field is a (nz+2) x (ny+2) x (nx+2) array, x fastest:
 *   element (i, j, k) at ((k * (ny+2)) + j) * (nx+2) + i.
 *   u lives on x-faces (i = 0..nx; i = 0, nx are the walls; i = nx+1 unused),
 *   v on y-faces, w on z-faces (cyclically); T at cell centres with one wall
 *   node per side (index 0 and n+1).  Entries that are not interior rows
 *   (walls, edges, padding) are part of the vector; operators write them with
 *   the values their definition gives (mostly 0).
 *
 * The discretisation is the second-order staggered finite-volume scheme with
 * stored wall nodes read from Sec. 3.1 of the paper; the equations are
 * eqs (1)-(3) in the Gr^1/2 scaling: nu = Gr^-1/2, kappa = nu / Pr, b = 1.
 */
#ifndef FVK_H
#define FVK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fvk_ctx fvk_ctx;

typedef enum {
    FVK_OK = 0,
    FVK_EINVAL = 1,      /* bad argument (size, enum, null pointer)           */
    FVK_ENOMEM = 2,      /* device or host allocation failed                  */
    FVK_EHIP = 3,        /* a HIP runtime call failed                         */
    FVK_ENOCONV = 4,     /* SIMPLE pass cap, GMRES/BiCGstab(2) or Newton limit */
    FVK_EBREAKDOWN = 5   /* Krylov breakdown (zero norm / NaN)                */
} fvk_status;

/* Spanwise (y = 0, 1) thermal walls: eq. (6) perfectly conducting, eq. (7)
 * perfectly insulated. */
typedef enum { FVK_SPAN_CC = 0, FVK_SPAN_AA = 1 } fvk_span_bc;

/* Face coordinates f_i = map(i / N): uniform; eq. (22) x - s sin(2 pi x)
 * (0 <= s < 1/(2 pi)); tanh clustering (1 + tanh(s (2x - 1)) / tanh s) / 2. */
typedef enum { FVK_GRID_UNIFORM = 0, FVK_GRID_SINE = 1, FVK_GRID_TANH = 2 } fvk_grid_kind;

/* FVK_FP64: everything in FP64.  FVK_MIXED: the Poisson eigenbasis
 * transforms of the SIMPLE pass run in FP32 (FP32 accumulation); the SIMPLE
 * loop repeats the pass (FP64 divergence, FP64 correction) as iterative
 * refinement until the divergence test passes.  Everything else is FP64. */
typedef enum { FVK_FP64 = 0, FVK_MIXED = 1 } fvk_prec;

/* ---------------------------------------------------------------- context */

/* Create a context for an nx x ny x nz finite-volume grid (each >= 2, each
 * <= 1024).  `s` is the stretching parameter of `grid_kind`.  Builds the grid,
 * the 1D eigendecompositions of eq. (15) (host, FP64) and allocates all
 * device workspace.  `hip_stream` is a hipStream_t (NULL = default stream).
 * On failure *out is NULL. */
fvk_status fvk_create(fvk_ctx **out, int nx, int ny, int nz, int grid_kind, double s,
                      int span_bc, double Gr, double Pr, int prec, void *hip_stream);
fvk_status fvk_destroy(fvk_ctx *ctx);
/* Later calls enqueue on hip_stream.  All calls share the context's
 * workspace, so the old stream is synchronised first (after reducing any
 * pending asynchronous divergence records, fvk_simple_stats, on it): a call
 * on the new stream never overlaps work still queued on the old one. */
fvk_status fvk_set_stream(fvk_ctx *ctx, void *hip_stream);
/* Re-derive nu = Gr^-1/2, kappa = nu / Pr, b = 1 (eqs (1)-(2)). */
fvk_status fvk_set_params(fvk_ctx *ctx, double Gr, double Pr);
/* Set the three coefficients directly (viscous scaling checks at Gr = 0,
 * derivative operators dA/dGr with b = 0). */
fvk_status fvk_set_coeffs(fvk_ctx *ctx, double nu, double kappa, double b);
/* Coupling terms of the linearised eqs (8)-(9) kept in the Jacobian (bit set)
 * or switched off (bit clear), for the mechanism experiment of Sec. 4.2
 * (terms nullified one at a time and the stability analysis rerun).  The
 * viscous and conductive terms are always kept; the residual (fv_residual) is
 * never affected.  Applies to fv_jacvec, simple_krylov_vec (forward and
 * transposed) and everything built on them -- newton_step included, so
 * restore FVK_TERMS_ALL before computing steady states.  Returns
 * FVK_EINVAL for bits outside FVK_TERMS_ALL. */
enum {
    FVK_TERM_BUOYANCY = 1 << 0,   /* T e_z in the momentum rows              */
    FVK_TERM_U_GRAD_V = 1 << 1,   /* (U.grad) v in the momentum rows         */
    FVK_TERM_V_GRAD_U = 1 << 2,   /* (v.grad) U in the momentum rows         */
    FVK_TERM_U_GRAD_T_X = 1 << 3, /* U dT/dx, V dT/dy, W dT/dz: energy rows  */
    FVK_TERM_U_GRAD_T_Y = 1 << 4,
    FVK_TERM_U_GRAD_T_Z = 1 << 5,
    FVK_TERM_V_GRAD_TH_X = 1 << 6, /* u dTheta/dx, v dTheta/dy, w dTheta/dz  */
    FVK_TERM_V_GRAD_TH_Y = 1 << 7,
    FVK_TERM_V_GRAD_TH_Z = 1 << 8,
    FVK_TERMS_ALL = (1 << 9) - 1
};
fvk_status fvk_set_terms(fvk_ctx *ctx, int mask);
/* Spectral shift of the Krylov operator for the eigenvalue problem of
 * eq. (10) (Sec. 3.1: rightmost eigenvalues by Arnoldi).  A = P J maps every
 * stored array into the constraint subspace S (divergence-free velocity,
 * homogeneous boundary values), so on whole arrays it has, besides the
 * spectrum of eq. (10) on S, the eigenvalue 0 with the multiplicity of the
 * complement ker P.  With sigma != 0, simple_krylov_vec (and arnoldi_step,
 * arnoldi_step_lagged, everything built on them) applies
 *     A_sigma = P (J + sigma I) = A + sigma P         (transpose = 0)
 *     A_sigma^T = J^T P^T + sigma P^T                 (transpose = 1)
 * whose spectrum is {lambda + sigma : lambda of eq. (10)} together with the
 * 0 of ker P: the Krylov spaces, Ritz vectors and residuals are those of
 * A - sigma (I - P), which moves the complement to -sigma, and the physical
 * eigenvalues are the Ritz values minus sigma.  The stencils add sigma times
 * the centre value they already hold: no extra memory traffic.  p_out then
 * accumulates the pressure of P (J + sigma I) x.  fv_jacvec, fvk_project,
 * fv_residual, fvk_linear_solve and newton_step are never shifted (the
 * linear solves switch it off for the duration of the call).  Default 0.
 * Returns FVK_EINVAL for a non-finite sigma. */
fvk_status fvk_set_shift(fvk_ctx *ctx, double sigma);
fvk_status fvk_get_shift(const fvk_ctx *ctx, double *sigma);
fvk_status fvk_set_precision(fvk_ctx *ctx, int prec);
/* Kernels of the TPF Poisson solve of the SIMPLE pass (Sec. 3.1, eqs
 * (16)-(18)); the result is the same up to rounding order.
 *   FVK_TPF_AUTO   (default) FVK_TPF_AXES;
 *   FVK_TPF_AXES   six launches, one per axis transform (and direction);
 *   FVK_TPF_PLANES three launches whose blocks hold one plane of the cell
 *                  array in LDS: the x and y forward transforms (with the
 *                  divergence formed from the faces) per z plane; the z
 *                  forward transform, the scaling and the z inverse per y
 *                  plane; the y and x inverse transforms per z plane.  Only
 *                  for 4 <= nx, ny, nz <= 128.  Measured slower than the
 *                  per-axis kernels at every size from 48^3 to 128^3 (one
 *                  block per plane keeps at most 128 of the 256 compute
 *                  units busy through a chain of dependent steps), so it is
 *                  never chosen automatically.
 * Returns FVK_EINVAL for an unknown value or FVK_TPF_PLANES on a grid it
 * does not fit.  fvk_get_tpf_path reports the kernels the solve runs
 * (FVK_TPF_AXES or FVK_TPF_PLANES). */
typedef enum { FVK_TPF_AUTO = 0, FVK_TPF_AXES = 1, FVK_TPF_PLANES = 2 } fvk_tpf_path;
fvk_status fvk_set_tpf_path(fvk_ctx *ctx, int path);
fvk_status fvk_get_tpf_path(const fvk_ctx *ctx, int *path);
/* SIMPLE loop control (Sec. 3.1): stop when max |D v| < tol (default 1e-9,
 * the paper's pointwise criterion), at most max_passes passes (default 10). */
fvk_status fvk_set_simple(fvk_ctx *ctx, double tol, int max_passes);
/* off[f] = offset (in doubles) of field f in a 4-field vector, field_len =
 * (nx+2)(ny+2)(nz+2), n_total = 4 * field_len. */
fvk_status fvk_layout(const fvk_ctx *ctx, size_t off[4], size_t *field_len, size_t *n_total);
/* Host copies of one axis (0 = x, 1 = y, 2 = z): faces[0..n], centres[0..n+1]
 * (wall nodes included), widths[0..n+1] (widths[i] = f[i] - f[i-1] for the
 * first half, mirrored exactly onto the second since every grid kind is
 * symmetric about 1/2; ends 0).  Any pointer may be NULL. */
fvk_status fvk_grid_axis(const fvk_ctx *ctx, int axis, double *faces, double *centres,
                         double *widths);
const char *fvk_last_error(const fvk_ctx *ctx);
/* Host utility used at context creation for eq. (15): eigenvalues lam[0..n)
 * and orthonormal eigenvectors (Q row-major n x n, column q for lam[q]) of the
 * symmetric tridiagonal matrix with diagonal diag[0..n) and off-diagonal
 * off[0..n-1), by the implicit QL algorithm.  Host pointers; no GPU needed. */
fvk_status fvk_tridiag_eig(int n, const double *diag, const double *off, double *lam, double *Q);

/* ------------------------------------------------------------- operators */

/* F(U, Theta): residual of the steady eqs (1)-(2) at interior rows (Sec. 3.1
 * Newton step 2), pressure omitted; other entries 0.  base = (U, V, W, Theta)
 * with the inhomogeneous wall values of eqs (4)-(7) in its wall nodes.
 * project != 0 returns P F (SIMPLE projection of the velocity part,
 * temperature projection of eq. (21) of the T part). */
fvk_status fv_residual(fvk_ctx *ctx, const double *base, double *F, int project);

/* y = J x: the Jacobian of F about `base` (eqs (8)-(9)) at interior rows,
 * other entries 0 (transpose = 0); y = J^T x, the Euclidean transpose over
 * all stored entries (transpose = 1).  x and y must not overlap. */
fvk_status fv_jacvec(fvk_ctx *ctx, const double *base, const double *x, double *y,
                     int transpose);

/* y = P x (transpose = 0): the SIMPLE projection of the velocity part
 * (eq. (13): divergence-free, homogeneous no-slip) and the temperature
 * projection of eq. (21) (homogeneous thermal BCs); y = P^T x (transpose = 1),
 * computed as W P W^-1 (W = face control volumes) with the fixed pass count
 * (one in FP64, two in mixed precision).  x == y is allowed. */
fvk_status fvk_project(fvk_ctx *ctx, const double *x, double *y, int transpose);

/* The next Krylov vector, eqs (11)-(13): y = A x = P J x (transpose = 0) or
 * y = A^T x = J^T P^T x (transpose = 1).  p_out (nullable, device, nx*ny*nz
 * doubles, cell order x fastest) receives the accumulated pressure
 * correction.  If `passes` or `max_div` is non-NULL the call synchronises and
 * reports the SIMPLE pass count and the final max |D v|; if both are NULL the
 * call is asynchronous and the divergence check is recorded on the device
 * (fvk_simple_stats).  Returns FVK_ENOCONV when the pass cap is hit.  In
 * FP64 one pass is exact up to rounding; in mixed precision asynchronous
 * calls run a fixed number of FP32 solves with FP64 refinement passes: the
 * number the first asynchronous forward mixed call of the context needed
 * (that call runs the adaptive loop synchronously; one more if its final
 * divergence came within a factor 10 of the tolerance; at least 2; reset by
 * fvk_set_simple; see fvk_mixed_passes), and every call's divergence test is
 * still recorded.  The transposed call always runs the fixed pass count (its
 * internal divergence, of W^-1 x, is reported but not tested and not
 * recorded).
 * x and y must not overlap. */
fvk_status simple_krylov_vec(fvk_ctx *ctx, const double *base, const double *x, double *y,
                             double *p_out, int transpose, int *passes, double *max_div);
/* The fixed pass count of asynchronous mixed-precision calls and whether it
 * has been calibrated by an adaptive call (see simple_krylov_vec). */
fvk_status fvk_mixed_passes(const fvk_ctx *ctx, int *passes, int *calibrated);
/* Visualisation of a 3D velocity field by divergence-free projections onto
 * the planes normal to one axis and their vector potentials (Sec. 3.2,
 * Psi_x, Psi_y, Psi_z).  For axis a (0 = x, 1 = y, 2 = z) with the in-plane
 * axes (b, c) in cyclic order: vproj (3 stored velocity fields, the layout
 * of the first three fields of a vector) = the W-orthogonal projection of
 * vel onto the fields with a zero a-component, zero wall entries and zero
 * in-plane divergence D_bc in every a-plane (one plane-wise TPF solve, the
 * 2D analogue of the SIMPLE step, FP64 whatever the context precision);
 * psi (nullable, one stored field) = the vector potential on the a-edges:
 * vproj = curl(psi e_a), i.e. vproj_b = d psi / d c, vproj_c = -d psi / d b,
 * psi = 0 on the walls; entry (i, j, k) holds the edge at cell index
 * (1..n_a) along a and face indices (0..n) along b and c, other entries 0.
 * vel may be a 4-field vector (its first three fields are read); vproj may
 * be vel.  Uses the context's Poisson workspace (stream-ordered). */
fvk_status fvk_psi_projection(fvk_ctx *ctx, const double *vel, int axis, double *vproj,
                              double *psi);
/* Largest max |D v| seen by asynchronous forward calls since the last query,
 * and the number of such calls that needed more passes than the fixed count.
 * Resets.  The device keeps each asynchronous call's block maxima and reduces
 * them 64 calls at a time; this call (and fvk_set_simple, fvk_set_stream)
 * reduces the pending ones first. */
fvk_status fvk_simple_stats(fvk_ctx *ctx, double *max_div, int *n_unconverged);

/* One Arnoldi step on A (or A^T): V holds j+1 orthonormal 4-field vectors
 * with leading dimension ldv (doubles, >= n_total) and room for vector j+1.
 * Computes w = A v_j, orthogonalises it against v_0..v_j by classical
 * Gram-Schmidt with one re-orthogonalisation pass, stores v_{j+1} = w/|w| and
 * writes h_col[0..j+1] (host): the new Hessenberg column with
 * h_col[j+1] = |w|.  Returns FVK_EBREAKDOWN if |w| vanishes (then v_{j+1}
 * is left unnormalised). */
fvk_status arnoldi_step(fvk_ctx *ctx, const double *base, double *V, size_t ldv, int j,
                        double *h_col, int transpose);

/* The same Arnoldi process (Sec. 3.1's Arnoldi iteration for the rightmost
 * eigenvalues of eq. (10)) with the re-orthogonalisation lagged by one step,
 * so that each step reads the basis twice instead of four times: one pass of
 * dot products against v_j and w, one pass of updates.
 * State between calls: V holds v_0..v_{j-1} (orthonormal) and, in slot j, a
 * vector that is orthogonal to them only to first order and not normalised;
 * row j of H refers to that raw vector.  Step j computes w = A (slot j)
 * normalised, re-orthogonalises slot j (it becomes v_j), corrects the earlier
 * columns of H for it, projects w against v_0..v_j (coefficients from the same
 * dot products) and stores the result, un-normalised, in slot j+1; column j of
 * H is written with H[j+1][j] = 1 (it refers to the raw slot j+1).
 * H: host, row-major, leading dimension ldh (columns, >= j+1), at least j+2
 * rows; rows 0..j and columns 0..j are read and written.  For j = 0 slot 0
 * holds the start vector (any norm) and row 0 of H is empty.  Returns
 * FVK_EBREAKDOWN if slot j is zero or lies in the span of v_0..v_{j-1} (the
 * Krylov space is invariant): then H is corrected with row j set to zero and
 * V is left as it was. */
fvk_status arnoldi_step_lagged(fvk_ctx *ctx, const double *base, double *V, size_t ldv, int j,
                               double *H, int ldh, int transpose);
/* The same step for an operator applied by the caller (a polynomial in A,
 * e.g. the Chebyshev filter of an accelerated Arnoldi iteration, Sec. 3.1's
 * Chebyshev-preconditioned eigenvalue solver): slot j+1 must already hold the
 * operator applied to slot j (the raw vector, as stored); everything else is
 * as in arnoldi_step_lagged. */
fvk_status arnoldi_step_lagged_applied(fvk_ctx *ctx, double *V, size_t ldv, int j, double *H,
                                       int ldh);
/* Completes a lagged Arnoldi sequence after step j-1: re-orthogonalises and
 * normalises slot j into v_j and corrects row j and the columns of H above it
 * (H as in arnoldi_step_lagged, columns 0..j-1).  Returns FVK_EBREAKDOWN as
 * above. */
fvk_status arnoldi_finish(fvk_ctx *ctx, double *V, size_t ldv, int j, double *H, int ldh);

/* ---------------------------------------------------------------- tracing */

/* Stages of the Krylov-vector path timed with HIP events on the context's
 * stream when tracing is on: the Jacobian stencil (forward or transposed,
 * including the fused temperature projection), the divergence of the momentum
 * predictor (on grids of at most 256 cells along x this is the first x-axis
 * transform of the solve, which forms the divergence as it reads its input),
 * the remaining axis transforms of the TPF Poisson solve (one event pair
 * around the back-to-back launches of a solve, counted as that many
 * launches), the velocity correction with its fused divergence check, and
 * the Gram-Schmidt kernels of arnoldi_step. */
enum { FVK_STAGE_JACVEC = 0, FVK_STAGE_DIV = 1, FVK_STAGE_TRANSFORM = 2, FVK_STAGE_CORRECT = 3,
       FVK_STAGE_ORTHO = 4, FVK_NSTAGES = 5 };
/* mask: bit s enables stage s (0 = off).  Each timed stage records two
 * events (a few microseconds of queue overhead each). */
fvk_status fvk_set_timing(fvk_ctx *ctx, int mask);
/* Synchronises, returns accumulated milliseconds and launch counts per stage
 * (host arrays of FVK_NSTAGES entries) since the last read, and resets. */
fvk_status fvk_timing_read(fvk_ctx *ctx, double *ms, int *counts);

/* ------------------------------------------------------- vector kernels */

/* out[q] = <V_q, w> for q < m over n doubles (host out). */
fvk_status fvk_multidot(fvk_ctx *ctx, const double *V, size_t ldv, int m, const double *w,
                        size_t n, double *out);
/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the dot products of fvk_multidot, out_dev[q] = <V_q, w> for q < m, written
 * to DEVICE memory (out_dev, m doubles) in stream order, without any
 * allocation, copy to the host or synchronisation.  The block partials live
 * in a static device array of 2 MiB per GPU (1024 blocks x 256 vectors),
 * held until the process ends and shared by every call on that GPU: calls
 * that overlap on one GPU (two streams, two contexts) race on it.  m must be
 * 1 .. 256 (FVK_EINVAL otherwise); ldv >= n when m > 1.  Same kernels and
 * summation order as fvk_multidot, so the results are identical. */
fvk_status fvk_multidot_noalloc(fvk_ctx *ctx, const double *V, size_t ldv, int m,
                                const double *w, size_t n, double *out_dev);
/* w <- alpha w + sum_q c[q] V_q (c host, m entries). */
fvk_status fvk_multiaxpy(fvk_ctx *ctx, double *w, double alpha, const double *V, size_t ldv,
                         int m, const double *c, size_t n);
/* z <- a x + b y + c z over n doubles (z must alias neither x nor y); the
 * three-term recurrence of polynomial filters, enqueued without any host
 * transfer. */
fvk_status fvk_lincomb3(fvk_ctx *ctx, double *z, double a, const double *x, double b,
                        const double *y, double c, size_t n);
/* y <- a x + b y over n doubles (x == y allowed: scaling). */
fvk_status fvk_axpby(fvk_ctx *ctx, double *y, double a, const double *x, double b, size_t n);
/* V[:, 0..k) <- V[:, 0..m) Q with Q host, column-major m x k (k <= m), in place
 * (Krylov-Schur restart / Ritz vector assembly). */
fvk_status fvk_basis_rotate(fvk_ctx *ctx, double *V, size_t ldv, int m, const double *Q, int k,
                            size_t n);

/* ----------------------------------------------------------------- Newton */

typedef struct {
    double tol;             /* stop when max |P F| < tol (default 1e-10)          */
    int gmres_m;            /* GMRES restart length (100, Sec. 3.1; 1 .. 400,
                               else FVK_EINVAL)                                   */
    int gmres_max_restarts; /* cap on GMRES(m) cycles per Newton step             */
    double sat_ratio;       /* GMRES saturated when a cycle reduces |r| by less
                               than this factor (0.9)                             */
    int bicgstab_max_it;    /* BiCGstab(2) iterations after GMRES (5000)           */
    double lin_tol;         /* relative residual target of the linear solve       */
    int max_newton;         /* Newton iterations per call                          */
} fvk_newton_opts;

typedef struct {
    double res_before, res_after;     /* max |P F| at entry / exit           */
    int newton_its, gmres_cycles, bicgstab_its, krylov_vecs;
    double lin_rel_res;               /* last linear relative residual       */
    int lin_status;                   /* fvk_status of the last linear solve */
} fvk_newton_report;

void fvk_newton_defaults(fvk_newton_opts *opts);
/* Solve A x = b (A = the Krylov operator about `base`, eqs (11)-(13)) for b in
 * the constraint subspace, from the initial x (device, in/out): restarted
 * GMRES(gmres_m) until |r|/|b| < lin_tol or saturation, then BiCGstab(2) from
 * the GMRES iterate (Sec. 3.1).  Uses opts->gmres_m, gmres_max_restarts,
 * sat_ratio, bicgstab_max_it and lin_tol; fills the linear fields of report
 * (lin_rel_res, lin_status, gmres_cycles, bicgstab_its, krylov_vecs).
 * The solution is returned projected onto the constraint subspace (one
 * fvk_project), which removes the gradient fields that rounding feeds into
 * the Krylov iterates.  BiCGstab(2) keeps its best iterate and stops when the
 * residual grows 1e4-fold over it or improves by less than 10% in 250
 * iterations.  Returns FVK_ENOCONV if lin_tol is not reached.
 * Allocates (gmres_m + 11) vectors of device workspace for the call. */
fvk_status fvk_linear_solve(fvk_ctx *ctx, const double *base, const double *b, double *x,
                            const fvk_newton_opts *opts, fvk_newton_report *report);
/* Newton iteration of Sec. 3.1 (steps 1-4) on `base` in place: b = P F;
 * solve A delta = b by restarted GMRES(m) until converged or saturated, then
 * BiCGstab(2) from the GMRES iterate, each linear solve to |r| <
 * max(lin_tol |b|, 0.01 tol) (Euclidean norms); base <- base - P delta (the correction
 * projected onto the constraint subspace, so D U stays at rounding level);
 * repeat up to max_newton times or until max |P F| < tol.  A linear solve that
 * misses lin_tol does not stop the iteration (its state is in the report);
 * returns FVK_ENOCONV if max |P F| >= tol after max_newton iterations.
 * report may be NULL. */
fvk_status newton_step(fvk_ctx *ctx, double *base, const fvk_newton_opts *opts,
                       fvk_newton_report *report);

#ifdef __cplusplus
}
#endif
#endif /* FVK_H */
