// Tensor-product-factorisation (TPF) Poisson solve of the SIMPLE pass
// (paper Sec. 3.1, eqs (16)-(18)):
//   phi = (E_x (x) E_y (x) E_z) Lambda^+ (E_x^-1 (x) E_y^-1 (x) E_z^-1) b,
//   Lambda_ijk = lx_i + ly_j + lz_k, the all-constant mode mapped to 0.
// Each factor is a dense N_a x N_a matrix applied along one axis of the compact
// (nz, ny, nx) cell array, i.e. a GEMM with N_a rows and the product of the
// other two extents as columns.  These are the only dense contractions of the
// method and run on the matrix cores: v_mfma_f64_16x16x4f64 in FP64 mode,
// v_mfma_f32_16x16x4f32 (FP32 inputs and accumulation) in mixed mode.
#include <algorithm>

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

// LDS-only workgroup barrier: orders LDS traffic without waiting for global
// loads or stores in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// Strip kernel: a block owns TN = 16 CT columns and ALL na output rows.  Its
// input strip (na x TN) is staged in LDS once (k-major, zero-padded to a
// multiple of 4 in K); the transform matrix M (at most 256 x 256, L2-resident
// and shared by every block) is streamed from global memory as MFMA
// A-fragments, so the K loop has no barriers.  Wave w owns the 16-row tiles
// w, w+4, w+8, ...  For the unit-stride axis the results are transposed
// through LDS so the stores are coalesced.
template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE, int CT, int MAXRT>
__global__ __launch_bounds__(NT) void k_axis_strip(const Tc *__restrict__ M, AxisView v,
                                                   const Tin *__restrict__ X,
                                                   Tout *__restrict__ Y,
                                                   const Tc *__restrict__ lamR,
                                                   const Tc *__restrict__ lam0,
                                                   const Tc *__restrict__ lam1) {
    constexpr int TN = 16 * CT;
    constexpr int LDX = TN + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Tc *sX = reinterpret_cast<Tc *>(smem_raw);
    typedef typename Mfma<Tc>::acc acc_t;
    const int na = v.na;
    const int Kp = (na + 3) & ~3;
    const int col0 = blockIdx.x * TN;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int e = tid; e < Kp * TN; e += NT) {
        int k, cc;
        if (CONTIG) {
            k = e % Kp;
            cc = e / Kp;
        } else {
            cc = e % TN;
            k = e / TN;
        }
        const int gc = col0 + cc;
        const bool ok = k < na && gc < v.ncols;
        const Tin val = X[col_addr(v, min(gc, v.ncols - 1)) + long(min(k, na - 1)) * v.sb];
        sX[k * LDX + cc] = ok ? Tc(val) : Tc(0);
    }
    __syncthreads();
    const int RT = (na + 15) >> 4;
    acc_t acc[MAXRT][CT];
#pragma unroll
    for (int q = 0; q < MAXRT; ++q)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[q][ct] = acc_t{0, 0, 0, 0};
    const int lr = lane & 15, lk = lane >> 4;
    // A-fragments stream from global memory through an AD-deep register ring
    // so AD loads per row tile are in flight while the MFMAs consume older ones
    constexpr int AD = 8;
    auto loadA = [&](int q, int k4) -> Tc {
        const int row = (wv + 4 * q) * 16 + lr;
        const int kk = k4 + lk;
        const Tc a0 = M[long(min(row, na - 1)) * na + min(kk, na - 1)];
        return (row < na && kk < na) ? a0 : Tc(0);
    };
    Tc ar[MAXRT][AD];
#pragma unroll
    for (int d = 0; d < AD; ++d)
#pragma unroll
        for (int q = 0; q < MAXRT; ++q) ar[q][d] = loadA(q, 4 * d);
    for (int kb4 = 0; kb4 < Kp; kb4 += 4 * AD) {
#pragma unroll
        for (int d = 0; d < AD; ++d) {
            const int k4 = kb4 + 4 * d;
            if (k4 < Kp) {
                const int kk = k4 + lk;
                Tc bfr[CT];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) bfr[ct] = sX[kk * LDX + ct * 16 + lr];
#pragma unroll
                for (int q = 0; q < MAXRT; ++q) {
                    if (wv + 4 * q < RT) {
#pragma unroll
                        for (int ct = 0; ct < CT; ++ct)
                            acc[q][ct] = Mfma<Tc>::op(ar[q][d], bfr[ct], acc[q][ct]);
                    }
                    ar[q][d] = loadA(q, k4 + 4 * AD);
                }
            }
        }
    }
    auto scaled = [&](Tc val, int row, int col) -> Tc {
        if (SCALE) {
            const Tc l = lamR[row] + lam0[col % v.n0] + lam1[col / v.n0];
            return (row == 0 && col == 0) ? Tc(0) : val / l;
        }
        return val;
    };
    if (!CONTIG) {
#pragma unroll
        for (int q = 0; q < MAXRT; ++q) {
            const int rt = wv + 4 * q;
            if (rt >= RT) continue;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = col0 + ct * 16 + lr;
                if (col >= v.ncols) continue;
                const long ca = col_addr(v, col);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rt * 16 + Mfma<Tc>::row(lane, r);
                    if (row < na) Y[ca + long(row) * v.sb] = Tout(scaled(acc[q][ct][r], row, col));
                }
            }
        }
        return;
    }
    // unit-stride axis: transpose through LDS ([col][row], pitch Kp + 1)
    __syncthreads();
    const int LDO = Kp + 1;
#pragma unroll
    for (int q = 0; q < MAXRT; ++q) {
        const int rt = wv + 4 * q;
        if (rt >= RT) continue;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rt * 16 + Mfma<Tc>::row(lane, r);
                if (row < Kp) sX[(ct * 16 + lr) * LDO + row] = acc[q][ct][r];
            }
    }
    __syncthreads();
    for (int e = tid; e < TN * na; e += NT) {
        const int cc = e / na, row = e % na;
        const int col = col0 + cc;
        if (col < v.ncols)
            Y[col_addr(v, col) + row] = Tout(scaled(sX[cc * LDO + row], row, col));
    }
}

template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE, int CT, int MAXRT>
void launch_strip(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR,
                  const Tc *l0, const Tc *l1, hipStream_t st) {
    const int Kp = (v.na + 3) & ~3;
    const size_t lds = std::max(size_t(Kp) * (16 * CT + 1), size_t(16 * CT) * (Kp + 1)) * sizeof(Tc);
    const int nb = (v.ncols + 16 * CT - 1) / (16 * CT);
    k_axis_strip<Tc, Tin, Tout, CONTIG, SCALE, CT, MAXRT><<<nb, NT, lds, st>>>(M, v, X, Y, lR, l0, l1);
}

template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE, int CT>
bool strip_dispatch(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR,
                    const Tc *l0, const Tc *l1, hipStream_t st) {
    const int rt = (v.na + 15) / 16;
    const int maxrt = (rt + 3) / 4;
    switch (maxrt) {
        case 1: launch_strip<Tc, Tin, Tout, CONTIG, SCALE, CT, 1>(M, v, X, Y, lR, l0, l1, st); return true;
        case 2: launch_strip<Tc, Tin, Tout, CONTIG, SCALE, CT, 2>(M, v, X, Y, lR, l0, l1, st); return true;
        case 3: launch_strip<Tc, Tin, Tout, CONTIG, SCALE, CT, 3>(M, v, X, Y, lR, l0, l1, st); return true;
        case 4: launch_strip<Tc, Tin, Tout, CONTIG, SCALE, CT, 4>(M, v, X, Y, lR, l0, l1, st); return true;
        default: return false;
    }
}

// GEMM-style transform: Y(P, T) = sum_K M[T][K] X(P, K) for every pencil P of
// the block's tile of 16 CP pencils and ALL transform outputs T (padded to
// 16 MAXRT per wave x 4 waves), so each input value is read from HBM once.
// Both operands stream through LDS in K-chunks of KC, double-buffered: the
// next chunk's global loads are in flight (in registers) while the MFMAs
// consume the current one; one barrier per chunk.  LDS tiles are K-major:
// sM[k][t], sX[k][p].  For the y/z axes the MFMA rows are T (A = M) and the
// 16 lanes of a result row are 16 consecutive pencils; for the unit-stride x
// axis (XAX) the roles swap (A = X, B = M^T) so the 16 lanes hold 16
// consecutive T -- contiguous -- and all stores are coalesced.
template <int MAXRT, int CP>
struct GemmTile {
    static constexpr int KC = 16;
    static constexpr int TT = 64 * MAXRT;          // T rows held (4 waves x MAXRT tiles)
    static constexpr int TP = 16 * CP;             // pencils per block
    static constexpr int LDT = TT + 1, LDP = TP + 1;
    static constexpr int NM = (TT * KC + NT - 1) / NT;   // M chunk entries per thread
    static constexpr int NX = (TP * KC + NT - 1) / NT;   // X chunk entries per thread
};

template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, int MAXRT, int CP>
__global__ __launch_bounds__(NT) void k_axis_gemm(const Tc *__restrict__ M, AxisView v,
                                                  const Tin *__restrict__ X,
                                                  Tout *__restrict__ Y,
                                                  const Tc *__restrict__ lamR,
                                                  const Tc *__restrict__ lam0,
                                                  const Tc *__restrict__ lam1) {
    typedef GemmTile<MAXRT, CP> G;
    constexpr int KC = G::KC, TT = G::TT, TP = G::TP, LDT = G::LDT, LDP = G::LDP;
    __shared__ Tc sM[2][KC * LDT];
    __shared__ Tc sX[2][KC * LDP];
    typedef typename Mfma<Tc>::acc acc_t;
    const int na = v.na;
    const int p0 = blockIdx.x * TP;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int nchunk = (na + KC - 1) / KC;
    Tc rm[G::NM], rx[G::NX];
    // global -> registers for chunk c (zero outside the matrix / pencil range)
    auto fetch = [&](int c) {
        const int kb = c * KC;
#pragma unroll
        for (int q = 0; q < G::NM; ++q) {
            const int e = tid + q * NT;
            const int t = e / KC, kk = e % KC;
            const bool ok = e < TT * KC && t < na && kb + kk < na;
            const Tc val = M[long(min(t, na - 1)) * na + min(kb + kk, na - 1)];
            rm[q] = ok ? val : Tc(0);
        }
#pragma unroll
        for (int q = 0; q < G::NX; ++q) {
            const int e = tid + q * NT;
            int p, kk;
            if (XAX) {
                p = e / KC;
                kk = e % KC;
            } else {
                kk = e / TP;
                p = e % TP;
            }
            const int gp = p0 + p, k = kb + kk;
            const bool ok = e < TP * KC && gp < v.ncols && k < na;
            const Tin val = X[col_addr(v, min(gp, v.ncols - 1)) + long(min(k, na - 1)) * v.sb];
            rx[q] = ok ? Tc(val) : Tc(0);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int q = 0; q < G::NM; ++q) {
            const int e = tid + q * NT;
            if (e < TT * KC) sM[buf][(e % KC) * LDT + e / KC] = rm[q];
        }
#pragma unroll
        for (int q = 0; q < G::NX; ++q) {
            const int e = tid + q * NT;
            if (e < TP * KC) {
                if (XAX)
                    sX[buf][(e % KC) * LDP + e / KC] = rx[q];
                else
                    sX[buf][(e / TP) * LDP + e % TP] = rx[q];
            }
        }
    };
    acc_t acc[MAXRT][CP];
#pragma unroll
    for (int q = 0; q < MAXRT; ++q)
#pragma unroll
        for (int cp = 0; cp < CP; ++cp) acc[q][cp] = acc_t{0, 0, 0, 0};
    fetch(0);
    put(0);
    lds_barrier();
    for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunk) fetch(c + 1);
#pragma unroll
        for (int k4 = 0; k4 < KC; k4 += 4) {
            const int kk = k4 + lk;
            Tc mf[MAXRT], xf[CP];
#pragma unroll
            for (int q = 0; q < MAXRT; ++q) mf[q] = sM[buf][kk * LDT + (wv + 4 * q) * 16 + lr];
#pragma unroll
            for (int cp = 0; cp < CP; ++cp) xf[cp] = sX[buf][kk * LDP + cp * 16 + lr];
#pragma unroll
            for (int q = 0; q < MAXRT; ++q)
#pragma unroll
                for (int cp = 0; cp < CP; ++cp)
                    acc[q][cp] = XAX ? Mfma<Tc>::op(xf[cp], mf[q], acc[q][cp])
                                     : Mfma<Tc>::op(mf[q], xf[cp], acc[q][cp]);
        }
        if (c + 1 < nchunk) put(buf ^ 1);
        lds_barrier();
    }
#pragma unroll
    for (int q = 0; q < MAXRT; ++q) {
        const int tb = (wv + 4 * q) * 16;
        if (tb >= na) continue;
#pragma unroll
        for (int cp = 0; cp < CP; ++cp)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int t, pp;
                if (XAX) {
                    t = tb + lr;
                    pp = p0 + cp * 16 + Mfma<Tc>::row(lane, r);
                } else {
                    t = tb + Mfma<Tc>::row(lane, r);
                    pp = p0 + cp * 16 + lr;
                }
                if (t >= na || pp >= v.ncols) continue;
                Tc val = acc[q][cp][r];
                if (SCALE) {
                    const Tc l = lamR[t] + lam0[pp % v.n0] + lam1[pp / v.n0];
                    val = (t == 0 && pp == 0) ? Tc(0) : val / l;
                }
                Y[col_addr(v, pp) + long(t) * v.sb] = Tout(val);
            }
    }
}

template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, int MAXRT, int CP>
void launch_gemm(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR,
                 const Tc *l0, const Tc *l1, hipStream_t st) {
    const int nb = (v.ncols + 16 * CP - 1) / (16 * CP);
    k_axis_gemm<Tc, Tin, Tout, XAX, SCALE, MAXRT, CP><<<nb, NT, 0, st>>>(M, v, X, Y, lR, l0, l1);
}

// pick the per-wave row tiles from the transform length (<= 256) and the
// pencils per block so the grid has enough blocks to fill the chip
template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE>
bool gemm_dispatch(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR,
                   const Tc *l0, const Tc *l1, hipStream_t st) {
    const int maxrt = ((v.na + 15) / 16 + 3) / 4;
    const bool cp2 = (v.ncols + 31) / 32 >= 1024;
#define FVK_GEMM_CASE(R)                                                                   \
    case R:                                                                                \
        if (cp2)                                                                           \
            launch_gemm<Tc, Tin, Tout, XAX, SCALE, R, 2>(M, v, X, Y, lR, l0, l1, st);      \
        else                                                                               \
            launch_gemm<Tc, Tin, Tout, XAX, SCALE, R, 1>(M, v, X, Y, lR, l0, l1, st);      \
        return true;
    switch (maxrt) {
        FVK_GEMM_CASE(1)
        FVK_GEMM_CASE(2)
        FVK_GEMM_CASE(3)
        FVK_GEMM_CASE(4)
        default:
            return false;
    }
#undef FVK_GEMM_CASE
}

template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE>
void run_axis(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR, const Tc *l0,
              const Tc *l1, hipStream_t st) {
    // strip kernel for transform lengths up to 256; one or two column tiles
    // per block depending on how many blocks that gives
    if (gemm_dispatch<Tc, Tin, Tout, CONTIG, SCALE>(M, v, X, Y, lR, l0, l1, st)) return;
    dim3 grid((v.ncols + TN - 1) / TN, (v.na + TM - 1) / TM);
    k_axis<Tc, Tin, Tout, CONTIG, SCALE><<<grid, NT, 0, st>>>(M, v, X, Y, lR, l0, l1);
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
    // one event pair around the six back-to-back launches
    timing_begin(ctx, FVK_STAGE_TRANSFORM);
    run_axis<Tc, double, Tc, true, false>(Einv[0], vx, b, t0, nullptr, nullptr, nullptr, st);
    run_axis<Tc, Tc, Tc, false, false>(Einv[1], vy, t0, t1, nullptr, nullptr, nullptr, st);
    run_axis<Tc, Tc, Tc, false, true>(Einv[2], vz, t1, t0, lam[2], lam[0], lam[1], st);
    run_axis<Tc, Tc, Tc, false, false>(E[2], vz, t0, t1, nullptr, nullptr, nullptr, st);
    run_axis<Tc, Tc, Tc, false, false>(E[1], vy, t1, t0, nullptr, nullptr, nullptr, st);
    run_axis<Tc, Tc, double, true, false>(E[0], vx, t0, phi, nullptr, nullptr, nullptr, st);
    timing_end(ctx, FVK_STAGE_TRANSFORM, 6);
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
