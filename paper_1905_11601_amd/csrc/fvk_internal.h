// Internal declarations of the fvk library (context, device geometry, kernel
// launchers).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fvk.h"

namespace fvk {

// Per-axis coefficient arrays on the device.  Each array has n+4 entries and
// the pointer is offset by one, so indices -1 .. n+2 are addressable; entries
// outside an array's valid range hold 0 (so reciprocals vanish there).
//   ih[i] = 1/h[i]           (i = 1..n)      cell widths
//   id[i] = 1/d[i]           (i = 0..n)      centre spacings
//   w[i]  = (f[i]-c[i])/d[i] (i = 0..n)      face interpolation weight
struct AxisDev {
    const double *ih, *id, *w;
};

struct Geo {
    int n[3];       // cells per axis
    int np[3];      // n + 2 (stored extent per axis)
    long s[3];      // strides: 1, np[0], np[0]*np[1]
    long F;         // field length
    AxisDev ax[3];
};

struct Coefs {
    double nu, kappa, b;
    // factors of the coupling terms of the linearised operator (1 kept, 0
    // switched off, fvk_set_terms): buoyancy, (U.grad) v, (v.grad) U, and per
    // axis U_a dT/dx_a and v_a dTheta/dx_a; `terms` is the bit mask
    double fb = 1.0, fuv = 1.0, fvu = 1.0, fut[3] = {1.0, 1.0, 1.0}, fvt[3] = {1.0, 1.0, 1.0};
    int terms = FVK_TERMS_ALL;
    // spectral shift of the Krylov operator (fvk_set_shift): the Jacobian
    // stencils of simple_krylov_vec return (J + sigma I) x, so the Krylov
    // vector becomes P (J + sigma I) x = (A + sigma P) x; 0 elsewhere
    double sigma = 0.0;
};

// Host-side description of one axis (natural indexing, see fvk.h).
struct AxisHost {
    int n = 0;
    std::vector<double> f, c, h, d, w;
};

// One-axis eigendecomposition of the Neumann operator D_aa = E diag(lam) E^-1
// (row-major n x n matrices), lam[0] = 0 is the constant mode.
struct Eig1D {
    int n = 0;
    std::vector<double> lam, E, Einv;
};

// Axes up to this many cells use the even/odd half-size transforms.
constexpr int kSymMax = 512;

// Even/odd half-size factors of the same eigenbasis (neumann_eig_sym):
// A = [Ae (ne x ne) | Ao (no x no)] forward, B = [Be | Bo] inverse, both
// row-major; lam permuted even modes first.
struct EigSym {
    int n = 0, ne = 0, no = 0;
    std::vector<double> lam, A, B;
};

// HIP-event stage timing (see fvk_set_timing).
struct Timing {
    int mask = 0;
    std::vector<hipEvent_t> ev;          // pool, pairs (start, stop)
    std::vector<int> stage;              // stage of each recorded pair
    std::vector<int> launches;           // kernel launches inside each pair
    size_t used = 0;                     // pairs recorded since the last harvest
    double ms[8] = {0};
    int count[8] = {0};
};

struct Workspace {
    double *geo = nullptr;          // packed AxisDev arrays
    double *div = nullptr;          // n cells (compact), also r/V in transposed passes
    double *phi = nullptr;          // n cells (compact) FP64 Poisson solution
    void *tb0 = nullptr, *tb1 = nullptr;   // transform ping-pong buffers (FP64 sized)
    double *E[3] = {}, *Einv[3] = {}, *lam[3] = {};
    float *E32[3] = {}, *Einv32[3] = {}, *lam32[3] = {};
    // even/odd half-size factors (axes with at most kSymMax cells)
    double *Ah[3] = {}, *Bh[3] = {}, *lamp[3] = {};
    float *Ah32[3] = {}, *Bh32[3] = {}, *lamp32[3] = {};
    double *vtmp = nullptr;         // 4-field scratch vector
    double *vtmp2 = nullptr;        // 4-field scratch vector (transposed SIMPLE)
    double *coef_dev = nullptr;     // small coefficient arrays copied from the host
    size_t coef_len = 0;
    double *red = nullptr;          // reduction scratch (partials)
    size_t red_len = 0;
    double *dev_scalars = nullptr;  // small device scalars (dot products, norms)
    // block maxima of |D v| of the last pass of asynchronous forward calls,
    // one row of correct_blocks per call, reduced kRing rows at a time (or when
    // the record is read, the stream or the tolerance changes)
    double *ring = nullptr;
    int ring_n = 0;
    int *dev_counters = nullptr;    // [0] async calls above tolerance, [1] block counter
    double *div_slots = nullptr;    // [0] max |D v| of the last pass, [1] running max (async)
    double *zeros = nullptr;        // max(nx, ny, nz) zeros (plane-wise solves)
    double *host_pinned = nullptr;  // pinned host staging for small reads
    size_t host_pinned_len = 0;
};

}  // namespace fvk

struct fvk_ctx {
    int n[3] = {0, 0, 0};
    int kind = 0;
    double s = 0.0;
    int bc = 0;
    double Gr = 0.0, Pr = 0.0;
    fvk::Coefs co{0.0, 0.0, 1.0};
    int prec = 0;
    hipStream_t stream = nullptr;
    double simple_tol = 1e-9;
    int simple_cap = 10;
    int mixed_passes = 2;           // fixed pass count of asynchronous mixed calls
    bool mixed_calibrated = false;  // mixed_passes set by an adaptive forward call
    double shift = 0.0;             // fvk_set_shift: Krylov operator A + shift P
    int tpf_path = 0;               // fvk_set_tpf_path (FVK_TPF_*)
    fvk::AxisHost ax[3];
    fvk::Eig1D eig[3];
    fvk::EigSym esym[3];
    fvk::Geo geo{};
    fvk::Workspace ws;
    fvk::Timing tm;
    size_t ncell = 0;
    std::string err;
};

namespace fvk {

// ---- tracing (capi.cpp): bracket one launch of `stage` with events
void timing_begin(fvk_ctx *ctx, int stage);
void timing_end(fvk_ctx *ctx, int stage, int launches = 1);

// ---- host utilities (eig.cpp)
void build_axis(AxisHost &a, int n, int kind, double s);
void neumann_eig(const AxisHost &a, Eig1D &e);
void neumann_eig_sym(const AxisHost &a, EigSym &e);
int tridiag_eig(int n, const double *diag, const double *off, double *lam, double *Q);

// ---- stencil kernels (kernels_stencil.hip); all enqueue on `st`
// y_v (3 fields) / y_T (1 field) = J x; ext != 0 applies Ext_T to the T part
void launch_jacvec(const Geo &g, Coefs c, int span_aa, int ext, const double *base,
                   const double *x, double *yv, double *yT, hipStream_t st);
void launch_jacvec_T(const Geo &g, Coefs c, int span_aa, int fold_ext, const double *base,
                     const double *yvel, const double *yT, double *x, hipStream_t st);
void launch_residual(const Geo &g, Coefs c, int span_aa, const double *base, double *F,
                     hipStream_t st);
void launch_div(const Geo &g, const double *v, double *div, hipStream_t st, bool win = false);
// v_out = v_in - G phi (wall entries 0), p_out += phi, div_out = D v_out (if non-null),
// block maxima of |D v_out| to red[0 .. correct_blocks)
void launch_correct_oop(const Geo &g, const double *vin, double *vout, const double *phi,
                        double *p_out, double *div_out, double *red, hipStream_t st,
                        bool win = false, bool wout = false);
int correct_blocks(const Geo &g);
// rows of the ring of asynchronous divergence records
constexpr int kRing = 64;
// for each of the n rows of nblk block maxima (in order): running[0] =
// max(running[0], row max), count_over[0] += (row max >= tol)
void launch_ring_reduce(const double *rows, int nblk, int n, double *running, int *count_over,
                        double tol, hipStream_t st);
// interior velocity faces scaled by W = d_A h_B h_C (inverse: by 1/W), rest 0
void launch_face_scale(const Geo &g, const double *src, double *dst, int inverse,
                       hipStream_t st);
void launch_ext_T(const Geo &g, int span_aa, const double *src, double *dst, hipStream_t st);
void launch_ext_T_T(const Geo &g, int span_aa, const double *src, double *dst, hipStream_t st);
void launch_zero_vel_walls(const Geo &g, const double *src, double *dst, hipStream_t st);

// ---- static scratch of the non-allocating entry point (noalloc.hip): looks
// up its device address on the current device once; false with a message on
// failure
bool noalloc_prepare(std::string *err);

// ---- TPF (kernels_tpf.hip)
// phi = L^+ b by the TPF transforms.  With vel != nullptr (only where
// tpf_fuses_div), b is not read: the right-hand side is D vel (win: D W^-1 vel)
// formed inside the first transform.
void tpf_solve(fvk_ctx *ctx, const double *b, double *phi, bool fp32, hipStream_t st,
               const double *vel = nullptr, int win = 0);
bool tpf_fuses_div(const fvk_ctx *ctx);
// the fused plane kernels (kernels_tpf_plane.hip): every axis 4 .. 128 cells
bool tpf_plane_fits(const int n[3]);
bool tpf_uses_planes(const fvk_ctx *ctx);
void tpf_solve_planes(fvk_ctx *ctx, const double *b, double *phi, bool fp32, hipStream_t st,
                      const double *vel, int win);
// phi = L_bc^+ b in every plane normal to axis `normal` (b, c the other two
// axes), FP64; the constant mode of each plane gets coefficient 0
void tpf_solve_plane(fvk_ctx *ctx, const double *b, double *phi, int normal, hipStream_t st);

// ---- plane projections (kernels_psi.hip)
// div = D_bc v at the cells (in-plane faces only; wall faces read as 0)
void launch_div_plane(const Geo &g, const double *v, double *div, int normal, hipStream_t st);
// vout = in-plane components of vin minus G_bc phi at interior faces, 0 elsewhere
// (normal component 0); vout may be vin
void launch_correct_plane(const Geo &g, const double *vin, const double *phi, double *vout,
                          int normal, hipStream_t st);
// psi (one stored field) on the edges along `normal`: v = curl(psi e_normal),
// 0 on the walls, by integration of the first in-plane component
void launch_psi_lines(const Geo &g, const double *vp, double *psi, int normal, hipStream_t st);

// ---- BLAS-like kernels (kernels_blas.hip)
int multidot_blocks(size_t n);
void launch_multidot(const double *V, size_t ldv, int m, const double *w, size_t n,
                     double *partials, int nblk, hipStream_t st);
int multidot2_blocks(size_t n);
void launch_multidot2(const double *V, size_t ldv, int m, const double *x, const double *y,
                      size_t n, double *partials, int nblk, double *out, hipStream_t st);
void launch_update2(double *x, double *y, const double *V, size_t ldv, int m, const double *a_dev,
                    const double *b_dev, double c1, double c2, double c3, size_t n,
                    hipStream_t st);
void launch_reduce_partials(const double *partials, int nblk, int m, double *out, int accumulate,
                            hipStream_t st);
void launch_multiaxpy(double *w, double alpha, double beta, const double *V, size_t ldv, int m,
                      const double *c_dev, size_t n, hipStream_t st);
void launch_basis_rotate(double *V, size_t ldv, int m, const double *Q_dev, int k, size_t n,
                         hipStream_t st);
void launch_max_reduce(const double *partials, int nblk, double *out, double *running,
                       int *count_over, double tol, hipStream_t st);
void launch_absmax(const double *x, size_t n, double *partials, int nblk, hipStream_t st);
void launch_scale_inv_sqrt(double *w, const double *nrm2, size_t n, hipStream_t st);
void launch_axpby(double *y, double a, const double *x, double b, size_t n, hipStream_t st);
void launch_fill(double *y, double v, size_t n, hipStream_t st);
// z = a x + b y + c z (z may alias neither x nor y)
void launch_lincomb3(double *z, double a, const double *x, double b, const double *y, double c,
                     size_t n, hipStream_t st);
void launch_copy(double *dst, const double *src, size_t n, hipStream_t st);
void launch_scale(double *w, double alpha, size_t n, hipStream_t st);

}  // namespace fvk
