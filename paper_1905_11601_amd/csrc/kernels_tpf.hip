// Tensor-product-factorisation (TPF) Poisson solve of the SIMPLE pass
// (paper Sec. 3.1, eqs (16)-(18)):
//   phi = (E_x (x) E_y (x) E_z) Lambda^+ (E_x^-1 (x) E_y^-1 (x) E_z^-1) b,
//   Lambda_ijk = lx_i + ly_j + lz_k, the all-constant mode mapped to 0.
// Each factor is a dense N_a x N_a matrix applied along one axis of the compact
// (nz, ny, nx) cell array, i.e. a GEMM with N_a rows and the product of the
// other two extents as columns.  These are the only dense contractions of the
// method and run on the matrix cores: v_mfma_f64_16x16x4f64 in FP64 mode,
// v_mfma_f32_16x16x4f32 (FP32 inputs and accumulation) in mixed mode.
#include <type_traits>
#include <algorithm>

#include "fvk_internal.h"
#include "tpf_common.h"
#include "xcd.h"

namespace fvk {

namespace {

using tpf::Mfma;
using tpf::lds_barrier;
using tpf::recip;

constexpr int TM = 32, TN = 64, KC = 16, NT = 256;

struct AxisView {
    int na;      // transform length (rows of M, K of the product)
    long sb;     // stride of the transform index
    int n0;      // extent of the fastest column index
    long s0, s1; // strides of the two column indices
    int ncols;   // n0 * n1
    unsigned long long m0;   // 2^40 / n0 + 1: c / n0 == (c * m0) >> 40 for c n0 < 2^40
};

inline AxisView axis_view(int na, long sb, int n0, long s0, long s1, int ncols) {
    return AxisView{na, sb, n0, s0, s1, ncols, (1ull << 40) / unsigned(n0) + 1};
}

// column c -> (c / n0, c % n0) by a multiply-shift (no integer division)
__device__ __forceinline__ int col_hi(const AxisView &v, int c) {
    return int((unsigned long long)(unsigned)c * v.m0 >> 40);
}
__device__ __forceinline__ long col_addr(const AxisView &v, int c) {
    const int hi = col_hi(v, c);
    return long(hi) * v.s1 + long(c - hi * v.n0) * v.s0;
}

// Y = M applied along one axis of X.  Block tile: TM output rows x TN
// columns; each of the 4 wavefronts owns a 16 x 32 sub-tile (two 16x16 MFMA
// accumulators).  K is staged through LDS in chunks of KC.  CONTIG: the
// transform index is the unit-stride one (x axis), so X tiles are loaded with
// consecutive threads along K.  SCALE: multiply each output by
// 1 / (lamR[row] + lam0[c0] + lam1[c1]), 0 where that sum vanishes: the
// eigenvalues are <= 0 with exactly 0 only for the constant mode of an axis,
// so these are the singular modes (the all-constant one of the 3D solve; one
// per plane when an axis's eigenvalues are replaced by zeros, as in the
// plane-wise 2D solves).
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
                const int ch = col_hi(v, col);
                const Tc l = lamR[row] + lam0[col - ch * v.n0] + lam1[ch];
                val = l == Tc(0) ? Tc(0) : val / l;   // singular (constant) modes -> 0
            }
            Y[ca + long(row) * v.sb] = Tout(val);
        }
    }
}

// Even/odd transform of a mirror-symmetric axis (the half-size factors of
// neumann_eig_sym).  A block computes all outputs of a tile of 16 CP pencils
// with NW wavefronts; wave w owns output rows [16 w, 16 w + 16) of BOTH
// halves, so NW = ceil(ne / 16) leaves at most 15 padded rows.  Both
// operands stream through LDS in K-chunks of KC, double-buffered (the next
// chunk's global loads are in flight in registers while the MFMAs consume the
// current one; one barrier per chunk).  Two products of half the order run
// side by side:
//   FWD: even = Ae (x_k + x_{N-1-k}), odd = Ao (x_k - x_{N-1-k}) (the middle
//        value x_m enters the last even column when N is odd); outputs are
//        stored even modes first, SCALE multiplies by the reciprocal of the
//        (permuted) eigenvalue sums;
//   INV: P = Be y_even, Q = Bo y_odd; x_t = P_t + Q_t, x_{N-1-t} = P_t - Q_t
//        (x_m = P_m for odd N); P and Q of a row sit in the same lane.
// Half the flops and half the matrix entries of the full transform.  For the
// unit-stride x axis (XAX) the MFMA roles swap (A = X, B = M^T) so that the
// 16 lanes of a result row hold 16 consecutive transform indices and the
// stores are coalesced.
template <int NW, int CP>
struct SymTile {
    static constexpr int KC = 16;
    static constexpr int NTT = 64 * NW;            // threads
    static constexpr int TT = 16 * NW;             // rows per half
    static constexpr int TP = 16 * CP;             // pencils per block
    static constexpr int LDT = TT + 1, LDP = TP + 1;
    static constexpr int NM = (TT * KC + NTT - 1) / NTT;
    static constexpr int NX = (TP * KC + NTT - 1) / NTT;
};

// The even/odd transform kernel (see SymTile).  DIV (x-axis forward only):
// the input is not an array of cell values but the velocity fields X (3
// stored fields, geometry dg); the value at cell
// (i, j, k) is the divergence D v there (DIV = 1) or D W^-1 v (DIV = 2, the
// transposed projection), formed from the six face values when the pencil is
// staged -- the divergence kernel and its array are skipped.
template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, bool FWD, int NW,
          int CP, int DIV = 0>
__global__ __launch_bounds__(64 * NW) void k_axis_sym(const Tc *__restrict__ M, AxisView v,
                                                      const Tin *__restrict__ X,
                                                      Tout *__restrict__ Y,
                                                      const Tc *__restrict__ lamR,
                                                      const Tc *__restrict__ lam0,
                                                      const Tc *__restrict__ lam1,
                                                      Geo dg = Geo{}) {
    static_assert(DIV == 0 || (XAX && FWD), "divergence input: x-axis forward transform");
    typedef SymTile<NW, CP> G;
    constexpr int KC = G::KC, TT = G::TT, TP = G::TP, LDT = G::LDT, LDP = G::LDP,
                  NTT = G::NTT;
    __shared__ Tc sM[2][2][KC * LDT];   // [buffer][even/odd]
    __shared__ Tc sX[2][2][KC * LDP];
    typedef typename Mfma<Tc>::acc acc_t;
    const int n = v.na, nh = n / 2, ne = n - nh, no = nh;
    const Tc *Me = M, *Mo = M + long(ne) * ne;
    // XCD-aware tile order: neighbouring pencil tiles share the cache lines a
    // row of the array straddles (rows of 100 cells are not multiples of 16),
    // so consecutive tiles go to the same XCD and its L2 serves the second
    const int p0 = int(xcd_remap(blockIdx.x, gridDim.x)) * TP;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int nchunk = (ne + KC - 1) / KC;
    // fetch only issues loads (raw values, clamped addresses); masking and the
    // even/odd fold happen in put, after the MFMAs of the current chunk
    Tc rme[G::NM], rmo[G::NM], rxa[G::NX], rxb[G::NX];
    // DIV: the six face values of both mirrored cells, raw
    constexpr int ND = DIV ? G::NX : 1;
    double fa[ND][6], fb[ND][6];
    // cell (i, j, k) of pencil column gp (x axis: columns = (k, j)) at x index kc
    auto face_loads = [&](int gp, int kc, double *f) {
        const int kz = col_hi(v, gp), jy = gp - kz * v.n0;
        tpf::cell_faces(dg, X, kc + 1, jy + 1, kz + 1, f);
    };
    auto face_div = [&](int gp, int kc, const double *f) -> double {
        const int kz = col_hi(v, gp), jy = gp - kz * v.n0;
        return tpf::cell_div<DIV ? DIV : 1>(dg, f, kc + 1, jy + 1, kz + 1);
    };
    auto fetch = [&](int c) {
        const int kb = c * KC;
#pragma unroll
        for (int q = 0; q < G::NM; ++q) {
            const int e = tid + q * NTT;
            const int t = e / KC, k = kb + e % KC;
            rme[q] = Me[long(min(t, ne - 1)) * ne + min(k, ne - 1)];
            rmo[q] = Mo[long(min(t, no - 1)) * no + min(k, no - 1)];
        }
#pragma unroll
        for (int q = 0; q < G::NX; ++q) {
            const int e = tid + q * NTT;
            const int p = XAX ? e / KC : e % TP, kk = XAX ? e % KC : e / TP;
            const int k = kb + kk;
            const long base = col_addr(v, min(p0 + p, v.ncols - 1));
            if (DIV) {
                const int kc = min(k, n - 1), gp = min(p0 + p, v.ncols - 1);
                face_loads(gp, kc, fa[DIV ? q : 0]);
                face_loads(gp, n - 1 - kc, fb[DIV ? q : 0]);
            } else if (FWD) {
                const int kc = min(k, n - 1);
                rxa[q] = Tc(X[base + long(kc) * v.sb]);
                rxb[q] = Tc(X[base + long(n - 1 - kc) * v.sb]);
            } else {
                rxa[q] = Tc(X[base + long(min(k, ne - 1)) * v.sb]);
                rxb[q] = Tc(X[base + long(ne + min(k, no - 1)) * v.sb]);
            }
        }
    };
    auto put = [&](int buf, int c) {
        const int kb = c * KC;
#pragma unroll
        for (int q = 0; q < G::NM; ++q) {
            const int e = tid + q * NTT;
            const int t = e / KC, k = kb + e % KC;
            if (e < TT * KC) {
                sM[buf][0][(e % KC) * LDT + t] = (t < ne && k < ne) ? rme[q] : Tc(0);
                sM[buf][1][(e % KC) * LDT + t] = (t < no && k < no) ? rmo[q] : Tc(0);
            }
        }
#pragma unroll
        for (int q = 0; q < G::NX; ++q) {
            const int e = tid + q * NTT;
            const int p = XAX ? e / KC : e % TP, kk = XAX ? e % KC : e / TP;
            const int k = kb + kk;
            if (e < TP * KC) {
                const bool in = p0 + p < v.ncols;
                Tc a, b;
                if (DIV) {
                    const int kc = min(k, n - 1), gp = min(p0 + p, v.ncols - 1);
                    rxa[q] = Tc(face_div(gp, kc, fa[DIV ? q : 0]));
                    rxb[q] = Tc(face_div(gp, n - 1 - kc, fb[DIV ? q : 0]));
                }
                if (FWD) {
                    a = k < no ? rxa[q] + rxb[q] : (k < ne ? rxa[q] : Tc(0));   // middle
                    b = k < no ? rxa[q] - rxb[q] : Tc(0);
                } else {
                    a = k < ne ? rxa[q] : Tc(0);
                    b = k < no ? rxb[q] : Tc(0);
                }
                sX[buf][0][kk * LDP + p] = in ? a : Tc(0);
                sX[buf][1][kk * LDP + p] = in ? b : Tc(0);
            }
        }
    };
    acc_t ae[CP], ao[CP];
#pragma unroll
    for (int cp = 0; cp < CP; ++cp) {
        ae[cp] = acc_t{0, 0, 0, 0};
        ao[cp] = acc_t{0, 0, 0, 0};
    }
    // SCALE: the eigenvalue sums of this lane's outputs, loaded before the K
    // loop (clamped indices) so the epilogue does not wait on a gather
    constexpr int NS = SCALE ? CP : 1;
    Tc s01[NS][4], sre[NS][4], sro[NS][4];
    if (SCALE) {
#pragma unroll
        for (int cp = 0; cp < NS; ++cp)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = min(wv * 16 + (XAX ? lr : Mfma<Tc>::row(lane, r)), ne - 1);
                const int pp = min(p0 + cp * 16 + (XAX ? Mfma<Tc>::row(lane, r) : lr),
                                   v.ncols - 1);
                const int ph = col_hi(v, pp);
                s01[cp][r] = lam0[pp - ph * v.n0] + lam1[ph];
                sre[cp][r] = lamR[t];
                sro[cp][r] = lamR[min(ne + t, n - 1)];
            }
    }
    fetch(0);
    put(0, 0);
    lds_barrier();
    const int tb = wv * 16;
    for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunk) fetch(c + 1);
#pragma unroll
        for (int k4 = 0; k4 < KC; k4 += 4) {
            const int kk = k4 + lk;
            const Tc me = sM[buf][0][kk * LDT + tb + lr];
            const Tc mo = sM[buf][1][kk * LDT + tb + lr];
#pragma unroll
            for (int cp = 0; cp < CP; ++cp) {
                const Tc xe = sX[buf][0][kk * LDP + cp * 16 + lr];
                const Tc xo = sX[buf][1][kk * LDP + cp * 16 + lr];
                ae[cp] = XAX ? Mfma<Tc>::op(xe, me, ae[cp]) : Mfma<Tc>::op(me, xe, ae[cp]);
                ao[cp] = XAX ? Mfma<Tc>::op(xo, mo, ao[cp]) : Mfma<Tc>::op(mo, xo, ao[cp]);
            }
        }
        if (c + 1 < nchunk) put(buf ^ 1, c + 1);
        lds_barrier();
    }
    if (tb >= ne) return;
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
            if (t >= ne || pp >= v.ncols) continue;
            const long base = col_addr(v, pp);
            const Tc pe = ae[cp][r], po = ao[cp][r];
            if (FWD) {
                Tc ve = pe, vo = po;
                if (SCALE) {
                    const Tc l01 = s01[SCALE ? cp : 0][r];
                    // the eigenvalue sum vanishes exactly on the singular
                    // (all-constant) modes: mapped to 0
                    const Tc den = sre[SCALE ? cp : 0][r] + l01;
                    ve = den == Tc(0) ? Tc(0) : pe * recip(den);
                    if (t < no) vo = po * recip(sro[SCALE ? cp : 0][r] + l01);
                }
                Y[base + long(t) * v.sb] = Tout(ve);
                if (t < no) Y[base + long(ne + t) * v.sb] = Tout(vo);
            } else {
                if (t < no) {
                    Y[base + long(t) * v.sb] = Tout(pe + po);
                    Y[base + long(n - 1 - t) * v.sb] = Tout(pe - po);
                } else {
                    Y[base + long(t) * v.sb] = Tout(pe);   // the middle (odd N)
                }
            }
        }
}

template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, bool FWD, int NW, int CP,
          int DIV = 0>
void launch_sym(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR,
                const Tc *l0, const Tc *l1, hipStream_t st, const Geo &dg = Geo{}) {
    const int nb = (v.ncols + 16 * CP - 1) / (16 * CP);
    k_axis_sym<Tc, Tin, Tout, XAX, SCALE, FWD, NW, CP, DIV>
        <<<nb, 64 * NW, 0, st>>>(M, v, X, Y, lR, l0, l1, dg);
}

// x-axis forward transform of the divergence of the velocity fields X (DIV as
// in k_axis_sym); returns false when the axis is not handled this way
template <typename Tc, int DIV>
bool run_sym_div(const Tc *M, const AxisView &v, const double *X, Tc *Y, const Geo &dg,
                 hipStream_t st) {
    const int ne = v.na - v.na / 2;
    const bool cp2 = (v.ncols + 31) / 32 >= 1024;
    const Tc *none = nullptr;
    // long FP64 axes: four pencil tiles per block share each factor chunk
    // (197 VGPRs, one block per CU as with two tiles): 188 instead of 195 us
    // at 256^3; one tile per block (two blocks per CU) measured 250 us
    if (std::is_same<Tc, double>::value && ne > 112 && (v.ncols + 63) / 64 >= 512) {
        launch_sym<Tc, double, Tc, true, false, true, 8, 4, DIV>(M, v, X, Y, none, none, none, st,
                                                                 dg);
        return true;
    }
#define FVK_DIV_CASE(W)                                                                    \
    case W:                                                                                \
        if (cp2)                                                                           \
            launch_sym<Tc, double, Tc, true, false, true, W, 2, DIV>(M, v, X, Y, none, none, \
                                                                     none, st, dg);        \
        else                                                                               \
            launch_sym<Tc, double, Tc, true, false, true, W, 1, DIV>(M, v, X, Y, none, none, \
                                                                     none, st, dg);        \
        return true;
    switch ((ne + 15) / 16) {
        FVK_DIV_CASE(1)
        FVK_DIV_CASE(2)
        FVK_DIV_CASE(3)
        FVK_DIV_CASE(4)
        FVK_DIV_CASE(5)
        FVK_DIV_CASE(6)
        FVK_DIV_CASE(7)
        FVK_DIV_CASE(8)
        default:
            return false;
    }
#undef FVK_DIV_CASE
}

// one wave per 16 rows of the half length ne = ceil(N/2) <= 256; two pencil
// tiles per block when that still leaves >= 1024 blocks
template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, bool FWD>
void run_sym(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR, const Tc *l0,
             const Tc *l1, hipStream_t st) {
    const int ne = v.na - v.na / 2;
    const int nw = (ne + 15) / 16;
    const bool cp2 = (v.ncols + 31) / 32 >= 1024;
#define FVK_SYM_CASE(W)                                                                    \
    case W:                                                                                \
        if (cp2)                                                                           \
            launch_sym<Tc, Tin, Tout, XAX, SCALE, FWD, W, 2>(M, v, X, Y, lR, l0, l1, st);  \
        else                                                                               \
            launch_sym<Tc, Tin, Tout, XAX, SCALE, FWD, W, 1>(M, v, X, Y, lR, l0, l1, st);  \
        return;
    switch (nw) {
        FVK_SYM_CASE(1)
        FVK_SYM_CASE(2)
        FVK_SYM_CASE(3)
        FVK_SYM_CASE(4)
        FVK_SYM_CASE(5)
        FVK_SYM_CASE(6)
        FVK_SYM_CASE(7)
        FVK_SYM_CASE(8)
        default:
            if (nw <= 12)
                launch_sym<Tc, Tin, Tout, XAX, SCALE, FWD, 12, 1>(M, v, X, Y, lR, l0, l1, st);
            else
                launch_sym<Tc, Tin, Tout, XAX, SCALE, FWD, 16, 1>(M, v, X, Y, lR, l0, l1, st);
            return;
    }
#undef FVK_SYM_CASE
}

// Register-resident variant of k_axis_sym for ne = ceil(N/2) <= 16 NW: wave w
// keeps its 16-row slices of Ae/Ao (or Be/Bo) for the whole K range in
// registers, loaded once, and the block walks over pencil tiles of 16
// (persistent grid).  Only the pencil data goes through LDS: the whole K
// extent of the next tile is fetched into registers while the MFMAs consume
// the current tile, then written to the other LDS buffer -- one barrier per
// tile.  K and the rows are padded to 16 NW with zeros.
template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, bool FWD, int NW>
__global__ __launch_bounds__(64 * NW) void k_axis_res(const Tc *__restrict__ M, AxisView v,
                                                      const Tin *__restrict__ X,
                                                      Tout *__restrict__ Y,
                                                      const Tc *__restrict__ lamR,
                                                      const Tc *__restrict__ lam0,
                                                      const Tc *__restrict__ lam1) {
    constexpr int NTT = 64 * NW, KP = 16 * NW, KS = KP / 4, LDP = 17;
    constexpr int NXT = KP * 16 / NTT;   // pencil values per thread and half (= 4)
    __shared__ Tc sX[2][2][KP * LDP];
    typedef typename Mfma<Tc>::acc acc_t;
    const int n = v.na, nh = n / 2, ne = n - nh, no = nh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int tb = wv * 16;
    const int ntiles = (v.ncols + 15) / 16;
    // this wave's rows of both factors: lane holds M[tb + lr][4 s + lk]
    Tc me[KS], mo[KS];
    {
        const Tc *Me = M, *Mo = M + long(ne) * ne;
        const int t = tb + lr;
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4) {
            const int k = 4 * s4 + lk;
            const Tc ve = Me[long(min(t, ne - 1)) * ne + min(k, ne - 1)];
            const Tc vo = Mo[long(min(t, no - 1)) * no + min(k, no - 1)];
            me[s4] = (t < ne && k < ne) ? ve : Tc(0);
            mo[s4] = (t < no && k < no) ? vo : Tc(0);
        }
    }
    // fetch only issues the loads (raw values, clamped addresses); the fold
    // and the masking happen in put, after the MFMAs of the current tile, so
    // the loads stay in flight meanwhile
    Tc ra[NXT], rb[NXT];
    auto pk = [&](int q, int &p, int &k) {
        const int e = tid + q * NTT;
        if (XAX) {
            p = e / KP;
            k = e % KP;
        } else {
            k = e / 16;
            p = e % 16;
        }
    };
    auto fetch = [&](int tile) {
#pragma unroll
        for (int q = 0; q < NXT; ++q) {
            int p, k;
            pk(q, p, k);
            const long base = col_addr(v, min(tile * 16 + p, v.ncols - 1));
            if (FWD) {
                const int kc = min(k, n - 1);
                ra[q] = Tc(X[base + long(kc) * v.sb]);
                rb[q] = Tc(X[base + long(n - 1 - kc) * v.sb]);
            } else {
                ra[q] = Tc(X[base + long(min(k, ne - 1)) * v.sb]);
                rb[q] = Tc(X[base + long(ne + min(k, no - 1)) * v.sb]);
            }
        }
    };
    auto put = [&](int buf, int tile) {
#pragma unroll
        for (int q = 0; q < NXT; ++q) {
            int p, k;
            pk(q, p, k);
            const bool in = tile * 16 + p < v.ncols;
            Tc a, b;
            if (FWD) {
                a = k < no ? ra[q] + rb[q] : (k < ne ? ra[q] : Tc(0));   // k == m: middle
                b = k < no ? ra[q] - rb[q] : Tc(0);
            } else {
                a = k < ne ? ra[q] : Tc(0);
                b = k < no ? rb[q] : Tc(0);
            }
            const int o = k * LDP + p;
            sX[buf][0][o] = in ? a : Tc(0);
            sX[buf][1][o] = in ? b : Tc(0);
        }
    };
    int tile = blockIdx.x;
    if (tile >= ntiles) return;   // uniform per block
    fetch(tile);
    put(0, tile);
    lds_barrier();
    int buf = 0;
    while (true) {
        const int next = tile + gridDim.x;
        if (next < ntiles) fetch(next);
        acc_t ae = {0, 0, 0, 0}, ao = {0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4) {
            const int kk = 4 * s4 + lk;
            const Tc xe = sX[buf][0][kk * LDP + lr];
            const Tc xo = sX[buf][1][kk * LDP + lr];
            ae = XAX ? Mfma<Tc>::op(xe, me[s4], ae) : Mfma<Tc>::op(me[s4], xe, ae);
            ao = XAX ? Mfma<Tc>::op(xo, mo[s4], ao) : Mfma<Tc>::op(mo[s4], xo, ao);
        }
        if (tb < ne) {
            const int p0 = tile * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int t, pp;
                if (XAX) {
                    t = tb + lr;
                    pp = p0 + Mfma<Tc>::row(lane, r);
                } else {
                    t = tb + Mfma<Tc>::row(lane, r);
                    pp = p0 + lr;
                }
                if (t >= ne || pp >= v.ncols) continue;
                const long base = col_addr(v, pp);
                const Tc pe = ae[r], po = ao[r];
                if (FWD) {
                    Tc ve = pe, vo = po;
                    if (SCALE) {
                        const int ph = col_hi(v, pp);
                    const Tc l01 = lam0[pp - ph * v.n0] + lam1[ph];
                        const Tc den = lamR[t] + l01;
                        ve = den == Tc(0) ? Tc(0) : pe * recip(den);
                        if (t < no) vo = po * recip(lamR[ne + t] + l01);
                    }
                    Y[base + long(t) * v.sb] = Tout(ve);
                    if (t < no) Y[base + long(ne + t) * v.sb] = Tout(vo);
                } else {
                    if (t < no) {
                        Y[base + long(t) * v.sb] = Tout(pe + po);
                        Y[base + long(n - 1 - t) * v.sb] = Tout(pe - po);
                    } else {
                        Y[base + long(t) * v.sb] = Tout(pe);   // the middle (odd N)
                    }
                }
            }
        }
        if (next >= ntiles) break;
        put(buf ^ 1, next);
        lds_barrier();
        buf ^= 1;
        tile = next;
    }
}

template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, bool FWD, int NW>
void launch_res(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR,
                const Tc *l0, const Tc *l1, hipStream_t st) {
    // a few resident blocks per compute unit (256 CUs), each walking tiles
    const int ntiles = (v.ncols + 15) / 16;
    const int per_cu = NW <= 4 ? 2 : 1;
    const int nb = std::min(ntiles, 256 * per_cu);
    k_axis_res<Tc, Tin, Tout, XAX, SCALE, FWD, NW><<<nb, 64 * NW, 0, st>>>(M, v, X, Y, lR, l0, l1);
}

// 96 < ne <= 128 (the MFMA-bound sizes), and in FP64 also 64 < ne <= 96:
// register-resident factors on a persistent grid (at 160 cells the streaming
// kernel's 1,600 blocks leave a third round of resident blocks nearly empty:
// 38.3 -> 34.5 us per FP64 transform; in FP32 the streaming kernel stays
// faster there); shorter axes (latency-bound) and longer ones: the streaming
// kernel
template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, bool FWD>
void run_half(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR,
              const Tc *l0, const Tc *l1, hipStream_t st) {
    const int ne = v.na - v.na / 2;
    constexpr bool f64 = std::is_same<Tc, double>::value;
    if (ne > 96 && ne <= 128)
        launch_res<Tc, Tin, Tout, XAX, SCALE, FWD, 8>(M, v, X, Y, lR, l0, l1, st);
    else if (f64 && ne > 80 && ne <= 96)
        launch_res<Tc, Tin, Tout, XAX, SCALE, FWD, 6>(M, v, X, Y, lR, l0, l1, st);
    else if (f64 && ne > 64 && ne <= 80)
        launch_res<Tc, Tin, Tout, XAX, SCALE, FWD, 5>(M, v, X, Y, lR, l0, l1, st);
    else
        run_sym<Tc, Tin, Tout, XAX, SCALE, FWD>(M, v, X, Y, lR, l0, l1, st);
}

// full-matrix transform (axes longer than kSymMax cells)
template <typename Tc, typename Tin, typename Tout, bool CONTIG, bool SCALE>
void run_axis(const Tc *M, const AxisView &v, const Tin *X, Tout *Y, const Tc *lR, const Tc *l0,
              const Tc *l1, hipStream_t st) {
    dim3 grid((v.ncols + TN - 1) / TN, (v.na + TM - 1) / TM);
    k_axis<Tc, Tin, Tout, CONTIG, SCALE><<<grid, NT, 0, st>>>(M, v, X, Y, lR, l0, l1);
}


// Factors of one axis: the even/odd halves when the axis has at most kSymMax
// cells, else the full matrices; lam in the matching mode order.
template <typename Tc>
struct AxisFactors {
    const Tc *fwd, *inv, *lam;
    bool sym;
};

template <typename Tc, typename Tin, typename Tout, bool XAX, bool SCALE, bool FWD>
void axis_step(const AxisFactors<Tc> &f, const AxisView &v, const Tin *X, Tout *Y,
               const Tc *lR, const Tc *l0, const Tc *l1, hipStream_t st) {
    if (f.sym)
        run_half<Tc, Tin, Tout, XAX, SCALE, FWD>(FWD ? f.fwd : f.inv, v, X, Y, lR, l0, l1, st);
    else
        run_axis<Tc, Tin, Tout, XAX, SCALE>(FWD ? f.fwd : f.inv, v, X, Y, lR, l0, l1, st);
}

template <typename Tc>
void tpf_typed(fvk_ctx *ctx, const double *b, double *phi, const AxisFactors<Tc> *F,
               hipStream_t st, const double *vel, int win) {
    const int nx = ctx->n[0], ny = ctx->n[1], nz = ctx->n[2];
    const long pl = long(nx) * ny;
    // axis x: rows i, columns (k, j); axis y: rows j, columns (k, i);
    // axis z: rows k, columns (j, i)
    const AxisView vx = axis_view(nx, 1, ny, nx, pl, ny * nz);
    const AxisView vy = axis_view(ny, nx, nx, 1, pl, nx * nz);
    const AxisView vz = axis_view(nz, pl, nx, 1, nx, nx * ny);
    Tc *t0 = static_cast<Tc *>(ctx->ws.tb0);
    Tc *t1 = static_cast<Tc *>(ctx->ws.tb1);
    const Tc *none = nullptr;
    // one event pair around the back-to-back transform launches; the x
    // transform that also forms the divergence counts as the divergence stage
    if (vel) {   // the caller checked tpf_fuses_div
        timing_begin(ctx, FVK_STAGE_DIV);
        if (win)
            run_sym_div<Tc, 2>(F[0].fwd, vx, vel, t0, ctx->geo, st);
        else
            run_sym_div<Tc, 1>(F[0].fwd, vx, vel, t0, ctx->geo, st);
        timing_end(ctx, FVK_STAGE_DIV);
        timing_begin(ctx, FVK_STAGE_TRANSFORM);
    } else {
        timing_begin(ctx, FVK_STAGE_TRANSFORM);
        axis_step<Tc, double, Tc, true, false, true>(F[0], vx, b, t0, none, none, none, st);
    }
    axis_step<Tc, Tc, Tc, false, false, true>(F[1], vy, t0, t1, none, none, none, st);
    axis_step<Tc, Tc, Tc, false, true, true>(F[2], vz, t1, t0, F[2].lam, F[0].lam, F[1].lam, st);
    axis_step<Tc, Tc, Tc, false, false, false>(F[2], vz, t0, t1, none, none, none, st);
    axis_step<Tc, Tc, Tc, false, false, false>(F[1], vy, t1, t0, none, none, none, st);
    axis_step<Tc, Tc, double, true, false, false>(F[0], vx, t0, phi, none, none, none, st);
    timing_end(ctx, FVK_STAGE_TRANSFORM, vel ? 5 : 6);
}

// The plane-wise solve L_bc^+ b of the planes normal to axis `normal`: the
// transforms of the two in-plane axes only, the normal axis's eigenvalues
// replaced by zeros in the scaling (so each plane's constant mode is the
// singular one, mapped to 0).  FP64.
void tpf_plane_typed(fvk_ctx *ctx, const double *b, double *phi, const AxisFactors<double> *F,
                     const double *zeros, int normal, hipStream_t st) {
    const int nx = ctx->n[0], ny = ctx->n[1], nz = ctx->n[2];
    const long pl = long(nx) * ny;
    const AxisView vx = axis_view(nx, 1, ny, nx, pl, ny * nz);
    const AxisView vy = axis_view(ny, nx, nx, 1, pl, nx * nz);
    const AxisView vz = axis_view(nz, pl, nx, 1, nx, nx * ny);
    double *t0 = static_cast<double *>(ctx->ws.tb0);
    double *t1 = static_cast<double *>(ctx->ws.tb1);
    const double *none = nullptr;
    if (normal == 0) {   // planes x = const: axes y, z
        axis_step<double, double, double, false, false, true>(F[1], vy, b, t0, none, none, none, st);
        axis_step<double, double, double, false, true, true>(F[2], vz, t0, t1, F[2].lam, zeros,
                                                             F[1].lam, st);
        axis_step<double, double, double, false, false, false>(F[2], vz, t1, t0, none, none, none,
                                                               st);
        axis_step<double, double, double, false, false, false>(F[1], vy, t0, phi, none, none, none,
                                                               st);
    } else if (normal == 1) {   // planes y = const: axes x, z
        axis_step<double, double, double, true, false, true>(F[0], vx, b, t0, none, none, none, st);
        axis_step<double, double, double, false, true, true>(F[2], vz, t0, t1, F[2].lam, F[0].lam,
                                                             zeros, st);
        axis_step<double, double, double, false, false, false>(F[2], vz, t1, t0, none, none, none,
                                                               st);
        axis_step<double, double, double, true, false, false>(F[0], vx, t0, phi, none, none, none,
                                                              st);
    } else {   // planes z = const: axes x, y (scaling on the y step: columns (k, i))
        axis_step<double, double, double, true, false, true>(F[0], vx, b, t0, none, none, none, st);
        axis_step<double, double, double, false, true, true>(F[1], vy, t0, t1, F[1].lam, F[0].lam,
                                                             zeros, st);
        axis_step<double, double, double, false, false, false>(F[1], vy, t1, t0, none, none, none,
                                                               st);
        axis_step<double, double, double, true, false, false>(F[0], vx, t0, phi, none, none, none,
                                                              st);
    }
}

}  // namespace

void tpf_solve_plane(fvk_ctx *ctx, const double *b, double *phi, int normal, hipStream_t st) {
    const Workspace &w = ctx->ws;
    AxisFactors<double> F[3];
    for (int a = 0; a < 3; ++a) {
        const bool sym = ctx->n[a] <= kSymMax;
        F[a] = {sym ? w.Ah[a] : w.Einv[a], sym ? w.Bh[a] : w.E[a], sym ? w.lamp[a] : w.lam[a], sym};
    }
    tpf_plane_typed(ctx, b, phi, F, w.zeros, normal, st);
}

bool tpf_fuses_div(const fvk_ctx *ctx) {
    // the streaming even/odd kernel, up to 256 cells along x (for 193..256
    // cells it replaces the register-resident transform: its six face values
    // per cell do not fit beside the resident factors)
    const int ne = ctx->n[0] - ctx->n[0] / 2;
    return ctx->n[0] <= kSymMax && ne <= 128;
}

bool tpf_uses_planes(const fvk_ctx *ctx) {
    return ctx->tpf_path == FVK_TPF_PLANES && tpf_plane_fits(ctx->n);
}

void tpf_solve(fvk_ctx *ctx, const double *b, double *phi, bool fp32, hipStream_t st,
               const double *vel, int win) {
    if (tpf_uses_planes(ctx)) {
        tpf_solve_planes(ctx, b, phi, fp32, st, vel, win);
        return;
    }
    const Workspace &w = ctx->ws;
    if (fp32) {
        AxisFactors<float> F[3];
        for (int a = 0; a < 3; ++a) {
            const bool sym = ctx->n[a] <= kSymMax;
            F[a] = {sym ? w.Ah32[a] : w.Einv32[a], sym ? w.Bh32[a] : w.E32[a],
                    sym ? w.lamp32[a] : w.lam32[a], sym};
        }
        tpf_typed<float>(ctx, b, phi, F, st, vel, win);
    } else {
        AxisFactors<double> F[3];
        for (int a = 0; a < 3; ++a) {
            const bool sym = ctx->n[a] <= kSymMax;
            F[a] = {sym ? w.Ah[a] : w.Einv[a], sym ? w.Bh[a] : w.E[a],
                    sym ? w.lamp[a] : w.lam[a], sym};
        }
        tpf_typed<double>(ctx, b, phi, F, st, vel, win);
    }
}

}  // namespace fvk
