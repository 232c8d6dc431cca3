// Device helpers shared by the TPF transform kernels (per-axis kernels in
// kernels_tpf.hip, fused plane kernels in kernels_tpf_plane.hip).
#pragma once

#include "fvk_internal.h"

namespace fvk {
namespace tpf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Operands (both types): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
// Result row of accumulator register r in lane l (column l % 16) differs:
// f64 places row 4 r + l / 16, f32 places row 4 (l / 16) + r (checked by an
// in-bounds probe on gfx950).
template <>
struct Mfma<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc op(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Mfma<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc op(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// LDS-only workgroup barrier: orders LDS traffic without waiting for global
// loads or stores in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// 1 / d to full double precision: hardware estimate + two Newton steps
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ float recip(float d) { return 1.0f / d; }

// The six face values of cell (i, j, k) (1-based, stored indexing) of the
// three velocity fields X: u at i and i-1, v at j and j-1, w at k and k-1.
// (Templated on the element type only so that kernels instantiated for other
// inputs still compile; the fields are FP64.)
template <typename T>
__device__ __forceinline__ void cell_faces(const Geo &g, const T *__restrict__ X, int i, int j,
                                           int k, double *f) {
    const long p = (long(k) * g.np[1] + j) * g.np[0] + i;
    f[0] = double(X[p]);
    f[1] = double(X[p - 1]);
    f[2] = double(X[g.F + p]);
    f[3] = double(X[g.F + p - g.s[1]]);
    f[4] = double(X[2 * g.F + p]);
    f[5] = double(X[2 * g.F + p - g.s[2]]);
}

// Divergence at cell (i, j, k) from its face values f (cell_faces): D v
// (DIV = 1), or D W^-1 v (DIV = 2: interior faces divided by their control
// volumes W = d_A h_B h_C, wall faces 0) for the transposed projection.
template <int DIV>
__device__ __forceinline__ double cell_div(const Geo &g, const double *f, int i, int j, int k) {
    const double hx = g.ax[0].ih[i], hy = g.ax[1].ih[j], hz = g.ax[2].ih[k];
    if (DIV == 1) return (f[0] - f[1]) * hx + (f[2] - f[3]) * hy + (f[4] - f[5]) * hz;
    const double up = i < g.n[0] ? f[0] * (g.ax[0].id[i] * hy * hz) : 0.0;
    const double um = i > 1 ? f[1] * (g.ax[0].id[i - 1] * hy * hz) : 0.0;
    const double vp = j < g.n[1] ? f[2] * (g.ax[1].id[j] * hz * hx) : 0.0;
    const double vm = j > 1 ? f[3] * (g.ax[1].id[j - 1] * hz * hx) : 0.0;
    const double wp = k < g.n[2] ? f[4] * (g.ax[2].id[k] * hx * hy) : 0.0;
    const double wm = k > 1 ? f[5] * (g.ax[2].id[k - 1] * hx * hy) : 0.0;
    return (up - um) * hx + (vp - vm) * hy + (wp - wm) * hz;
}

}  // namespace tpf
}  // namespace fvk
