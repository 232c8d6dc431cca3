// Tensor-product-factorisation (TPF) Poisson solve of the SIMPLE pass
// (paper Sec. 3.1, eqs (16)-(18)):
//   phi = (E_x (x) E_y (x) E_z) Lambda^+ (E_x^-1 (x) E_y^-1 (x) E_z^-1) b,
//   Lambda_ijk = lx_i + ly_j + lz_k, the all-constant mode mapped to 0.
// Each factor is a dense N_a x N_a matrix applied along one axis of the compact
// (nz, ny, nx) cell array, i.e. a GEMM with N_a rows and the product of the
// other two extents as columns.  These are the only dense contractions of the
// method and run on the matrix cores: v_mfma_f64_16x16x4f64 in FP64 mode,
// v_mfma_f32_16x16x4f32 (FP32 inputs and accumulation) in mixed mode.
#include "fvk_internal.h"

namespace fvk {

namespace {

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

constexpr int TM = 32, TN = 64, KC = 16, NT = 256;

struct AxisView {
    int na;      // transform length (rows of M, K of the product)
    long sb;     // stride of the transform index
    int n0;      // extent of the fastest column index
    long s0, s1; // strides of the two column indices
    int ncols;   // n0 * n1
};

__device__ __forceinline__ long col_addr(const AxisView &v, int c) {
    return long(c / v.n0) * v.s1 + long(c % v.n0) * v.s0;
}

// Y = M applied along one axis of X.  Block tile: TM output rows x TN
// columns; each of the 4 wavefronts owns a 16 x 32 sub-tile (two 16x16 MFMA
// accumulators).  K is staged through LDS in chunks of KC.  CONTIG: the
// transform index is the unit-stride one (x axis), so X tiles are loaded with
// consecutive threads along K.  SCALE: multiply each output by
// 1 / (lamR[row] + lam0[c0] + lam1[c1]) (0 for the all-constant mode).
template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE>
__global__ __launch_bounds__(NT) void k_axis(const Tc *__restrict__ M, AxisView v,
                                             const Tin *__restrict__ X, Tout *__restrict__ Y,
                                             const Tc *__restrict__ lamR,
                                             const Tc *__restrict__ lam0,
                                             const Tc *__restrict__ lam1) {
    __shared__ Tc sM[TM][KC + 1];
    __shared__ Tc sX[KC][TN + 1];
    typedef typename Mfma<Tc>::acc acc_t;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
    const int wr = (wv >> 1) * 16, wc = (wv & 1) * 32;
    acc_t a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
    const int na = v.na;
    for (int kb = 0; kb < na; kb += KC) {
        for (int e = tid; e < TM * KC; e += NT) {
            const int r = e / KC, kk = e % KC;
            const int gr = row0 + r, gk = kb + kk;
            sM[r][kk] = (gr < na && gk < na) ? M[long(gr) * na + gk] : Tc(0);
        }
        for (int e = tid; e < KC * TN; e += NT) {
            int kk, cc;
            if (CONTIG) {
                kk = e % KC;
                cc = e / KC;
            } else {
                cc = e % TN;
                kk = e / TN;
            }
            const int gk = kb + kk, gc = col0 + cc;
            Tc val = Tc(0);
            if (gk < na && gc < v.ncols) val = Tc(X[col_addr(v, gc) + long(gk) * v.sb]);
            sX[kk][cc] = val;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < KC; k4 += 4) {
            const Tc a = sM[wr + (lane & 15)][k4 + (lane >> 4)];
            const Tc b0 = sX[k4 + (lane >> 4)][wc + (lane & 15)];
            const Tc b1 = sX[k4 + (lane >> 4)][wc + 16 + (lane & 15)];
            a0 = Mfma<Tc>::op(a, b0, a0);
            a1 = Mfma<Tc>::op(a, b1, a1);
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const acc_t acc = t ? a1 : a0;
        const int col = col0 + wc + t * 16 + (lane & 15);
        if (col >= v.ncols) continue;
        const long ca = col_addr(v, col);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + wr + Mfma<Tc>::row(lane, r);
            if (row >= na) continue;
            Tc val = acc[r];
            if (SCALE) {
                const Tc l = lamR[row] + lam0[col % v.n0] + lam1[col / v.n0];
                val = (row == 0 && col == 0) ? Tc(0) : val / l;
            }
            Y[ca + long(row) * v.sb] = Tout(val);
        }
    }
}

template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE>
void run_axis(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR, const Tc *l0,
              const Tc *l1, hipStream_t st) {
    dim3 grid((v.ncols + TN - 1) / TN, (v.na + TM - 1) / TM);
    k_axis<Tc, Tin, Tout, CONTIG, SCALE><<<grid, NT, 0, st>>>(M, v, X, Y, lR, l0, l1);
}

template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE>
void timed_axis(fvk_ctx *ctx, const Tc *M, const AxisView &v, const Tin *X, Tout *Y,
                const Tc *lR, const Tc *l0, const Tc *l1, hipStream_t st) {
    timing_begin(ctx, FVK_STAGE_TRANSFORM);
    run_axis<Tc, Tin, Tout, CONTIG, SCALE>(M, v, X, Y, lR, l0, l1, st);
    timing_end(ctx, FVK_STAGE_TRANSFORM);
}

template <typename Tc>
void tpf_typed(fvk_ctx *ctx, const double *b, double *phi, const Tc *const *E,
               const Tc *const *Einv, const Tc *const *lam, hipStream_t st) {
    const int nx = ctx->n[0], ny = ctx->n[1], nz = ctx->n[2];
    const long pl = long(nx) * ny;
    // axis x: rows i, columns (k, j); axis y: rows j, columns (k, i);
    // axis z: rows k, columns (j, i)
    const AxisView vx{nx, 1, ny, nx, pl, ny * nz};
    const AxisView vy{ny, nx, nx, 1, pl, nx * nz};
    const AxisView vz{nz, pl, nx, 1, nx, nx * ny};
    Tc *t0 = static_cast<Tc *>(ctx->ws.tb0);
    Tc *t1 = static_cast<Tc *>(ctx->ws.tb1);
    timed_axis<Tc, double, Tc, true, false>(ctx, Einv[0], vx, b, t0, nullptr, nullptr, nullptr, st);
    timed_axis<Tc, Tc, Tc, false, false>(ctx, Einv[1], vy, t0, t1, nullptr, nullptr, nullptr, st);
    timed_axis<Tc, Tc, Tc, false, true>(ctx, Einv[2], vz, t1, t0, lam[2], lam[0], lam[1], st);
    timed_axis<Tc, Tc, Tc, false, false>(ctx, E[2], vz, t0, t1, nullptr, nullptr, nullptr, st);
    timed_axis<Tc, Tc, Tc, false, false>(ctx, E[1], vy, t1, t0, nullptr, nullptr, nullptr, st);
    timed_axis<Tc, Tc, double, true, false>(ctx, E[0], vx, t0, phi, nullptr, nullptr, nullptr, st);
}

}  // namespace

void tpf_solve(fvk_ctx *ctx, const double *b, double *phi, bool fp32, hipStream_t st) {
    if (fp32) {
        const float *E[3] = {ctx->ws.E32[0], ctx->ws.E32[1], ctx->ws.E32[2]};
        const float *Ei[3] = {ctx->ws.Einv32[0], ctx->ws.Einv32[1], ctx->ws.Einv32[2]};
        const float *L[3] = {ctx->ws.lam32[0], ctx->ws.lam32[1], ctx->ws.lam32[2]};
        tpf_typed<float>(ctx, b, phi, E, Ei, L, st);
    } else {
        const double *E[3] = {ctx->ws.E[0], ctx->ws.E[1], ctx->ws.E[2]};
        const double *Ei[3] = {ctx->ws.Einv[0], ctx->ws.Einv[1], ctx->ws.Einv[2]};
        const double *L[3] = {ctx->ws.lam[0], ctx->ws.lam[1], ctx->ws.lam[2]};
        tpf_typed<double>(ctx, b, phi, E, Ei, L, st);
    }
}

}  // namespace fvk
