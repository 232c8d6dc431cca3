// Fused TPF solve for grids of at most 128 cells per axis (paper Sec. 3.1,
// eqs (16)-(18)): the six axis transforms of the solve run as three launches
// whose blocks each hold one whole plane of the cell array in LDS:
//
//   k_plane_fwd   one block per z plane (j, i): the right-hand side (or the
//                 divergence formed from the face values), x forward and y
//                 forward transforms;
//   k_plane_mid   one block per y plane (k, i): z forward transform, the
//                 scaling by 1 / (lx_i + ly_j + lz_k) (0 on the singular
//                 all-constant mode), z inverse transform;
//   k_plane_inv   one block per z plane: y inverse and x inverse transforms.
//
// At these sizes a per-axis launch is bound by memory latency, not by
// bandwidth or the matrix cores (8-16 MB per launch, 12 us per launch at 100^3
// for a few us of traffic); the plane kernels touch HBM once per plane and
// launch half as often, but one block per plane keeps at most 128 compute
// units busy, each through a chain of dependent load / transform / transform
// / store steps, and they measured slower than the per-axis kernels (41 + 2 x
// 36 us against 17 + 5 x 12 us per solve at 100^3): selectable
// (fvk_set_tpf_path), never chosen automatically.  Each transform is the even/odd pair of half-size
// products of the mirror-symmetric axis (the factors of neumann_eig_sym) on
// the matrix cores, with the operands read straight from the LDS plane and
// the factor slices of a wave held in registers.
//
// In LDS a plane is stored row-major with leading dimension nx + 1; x is the
// column index of every plane.  Forward inputs are folded in place: position
// k holds x_k + x_{N-1-k} and position N-1-k holds x_k - x_{N-1-k} (k < N/2;
// the middle value of an odd N stays).  Transform outputs are stored with the
// even modes first, as the per-axis kernels store them, so the permuted
// eigenvalue arrays index them directly.
#include <type_traits>

#include "fvk_internal.h"
#include "tpf_common.h"

namespace fvk {

namespace {

using tpf::Mfma;
using tpf::lds_barrier;
using tpf::recip;

constexpr int PW = 8;                         // waves per block
constexpr int PNT = 64 * PW;                  // threads per block
constexpr int PMAX = 128;                     // cells per axis
constexpr int PCAP = PMAX * (PMAX + 1);       // LDS plane capacity (elements)
constexpr int KSMAX = (PMAX / 2 + 3) / 4;     // K steps of 4 for a half of <= 64
constexpr int UMAX = 4;                       // output tiles per wave and half

template <typename Tc>
struct PlaneAxes {
    const Tc *fwd[3], *inv[3], *lam[3];   // half-size factors, permuted eigenvalues
    int n[3];
};

// The output tiles a wave computes in one transform of length n over npen
// pencils: rows [tb, tb + 16) of both halves, pencil tiles pt0, pt0 + dpt, ...
// (nu of them; 0 when the wave idles because PW is not a multiple of the
// number of row tiles).
struct Units {
    int tb, pt0, dpt, nu;
};

__device__ __forceinline__ Units units_of(int n, int npen, int wv) {
    const int ne = n - n / 2;
    const int tt = (ne + 15) / 16;          // row tiles per half (<= 4)
    const int wpt = PW / tt;                // waves per row tile (>= 2)
    const int npt = (npen + 15) / 16;       // pencil tiles (<= 8)
    Units u{0, 0, 1, 0};
    if (wv >= wpt * tt) return u;
    u.tb = (wv % tt) * 16;
    u.pt0 = wv / tt;
    u.dpt = wpt;
    u.nu = u.pt0 < npt ? (npt - u.pt0 + wpt - 1) / wpt : 0;
    return u;
}

// One even/odd transform on the LDS plane P.  ROW: the transform runs along
// the columns of each row (pencils = rows, the x axis); else along the rows
// of each column (pencils = columns).  FWD reads the folded input (even
// input k at position k, odd input k at N-1-k), the inverse reads the even
// modes at 0 .. ne-1 and the odd modes at ne .. N-1.  M: the ne x ne even
// factor followed by the no x no odd one, row-major.
//   result, COL: lane l, register r of tile q holds the output row
//     t = tb + row(l, r) of pencil p = pb_q + l % 16;
//   result, ROW: pencil p = pb_q + row(l, r), output row t = tb + l % 16
// (A = M, B = plane for columns; A = plane^T, B = M^T for rows, so the lanes
// of a result row always run along the contiguous x index).
template <typename Tc, bool ROW, bool FWD>
__device__ __forceinline__ void plane_transform(const Tc *P, int LD, int n, int npen,
                                                const Tc *__restrict__ M, const Units &u,
                                                int lane, typename Mfma<Tc>::acc (&ae)[UMAX],
                                                typename Mfma<Tc>::acc (&ao)[UMAX]) {
    const int ne = n - n / 2, no = n / 2;
    const int lr = lane & 15, lk = lane >> 4;
    const int t = u.tb + lr;
    const Tc *Me = M, *Mo = M + ne * ne;
    // this lane's factor entries M[t][4 s + lk] for every K step, 0 outside
    // (the same registers serve as A operand for columns and B for rows)
    // (one base address per half and immediate offsets: masked loads rather
    // than clamped indices, whose 64-bit addresses would stay live)
    Tc fe[KSMAX], fo[KSMAX];
    const Tc *re = Me + min(t, ne - 1) * ne + lk;
    const Tc *ro = Mo + min(t, no - 1) * no + lk;
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) {
        const int k = 4 * s + lk;
        fe[s] = Tc(0);
        fo[s] = Tc(0);
        if (t < ne && k < ne) fe[s] = re[4 * s];
        if (t < no && k < no) fo[s] = ro[4 * s];
    }
#pragma unroll
    for (int q = 0; q < UMAX; ++q) {
        ae[q] = typename Mfma<Tc>::acc{0, 0, 0, 0};
        ao[q] = typename Mfma<Tc>::acc{0, 0, 0, 0};
    }
    const int ks = (ne + 3) / 4;
    // operands of K step s from the plane; clamped positions hold finite
    // plane values and the factor entry is 0 there, so they add nothing
    auto load = [&](int s, Tc (&xe)[UMAX], Tc (&xo)[UMAX]) {
        const int k = 4 * s + lk;
        const int pe = min(k, ne - 1);
        const int po = FWD ? n - 1 - min(k, no - 1) : ne + min(k, no - 1);
#pragma unroll
        for (int q = 0; q < UMAX; ++q) {
            const int p = min((u.pt0 + q * u.dpt) * 16 + lr, npen - 1);
            xe[q] = ROW ? P[p * LD + pe] : P[pe * LD + p];
            xo[q] = ROW ? P[p * LD + po] : P[po * LD + p];
        }
    };
    // the operands of step s + 1 are read while the products of step s run;
    // the scheduling barrier keeps the compiler from hoisting every step's
    // reads to the top (they would not fit in registers)
    Tc xe[UMAX], xo[UMAX], ye[UMAX], yo[UMAX];
    load(0, xe, xo);
#pragma unroll
    for (int s = 0; s < KSMAX; ++s) {
        if (s < ks) {
            if (s + 1 < ks) load(s + 1, ye, yo);
#pragma unroll
            for (int q = 0; q < UMAX; ++q) {
                if (q < u.nu) {
                    ae[q] = ROW ? Mfma<Tc>::op(xe[q], fe[s], ae[q])
                                : Mfma<Tc>::op(fe[s], xe[q], ae[q]);
                    ao[q] = ROW ? Mfma<Tc>::op(xo[q], fo[s], ao[q])
                                : Mfma<Tc>::op(fo[s], xo[q], ao[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < UMAX; ++q) {
                xe[q] = ye[q];
                xo[q] = yo[q];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// In-place fold of the forward input along the columns of each of nr rows
// (the row transform's axis, length n) ...
template <typename Tc>
__device__ __forceinline__ void fold_rows(Tc *P, int LD, int n, int nr, int tid) {
    const int no = n / 2;
    for (int e = tid; e < nr * no; e += PNT) {
        const int r = e / no, k = e - r * no;
        Tc *row = P + r * LD;
        const Tc a = row[k], b = row[n - 1 - k];
        row[k] = a + b;
        row[n - 1 - k] = a - b;
    }
}
// ... and along the rows of each of nc columns (axis length n)
template <typename Tc>
__device__ __forceinline__ void fold_cols(Tc *P, int LD, int n, int nc, int tid) {
    const int no = n / 2;
    for (int e = tid; e < no * nc; e += PNT) {
        const int k = e / nc, c = e - k * nc;
        const Tc a = P[k * LD + c], b = P[(n - 1 - k) * LD + c];
        P[k * LD + c] = a + b;
        P[(n - 1 - k) * LD + c] = a - b;
    }
}

// Stage rows x nx values into the plane, value(r, c) read through `get`; LB
// elements per thread are loaded before any is stored, so their loads are in
// flight together.
template <int LB, typename Tc, typename Get>
__device__ __forceinline__ void stage_plane(Tc *P, int LD, int nr, int nc, int tid, Get get) {
    const int total = nr * nc;
    for (int e0 = 0; e0 < total; e0 += LB * PNT) {
        Tc v[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = min(e0 + q * PNT + tid, total - 1);
            const int r = e / nc;
            v[q] = get(r, e - r * nc);
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = e0 + q * PNT + tid;
            if (e < total) {
                const int r = e / nc;
                P[r * LD + (e - r * nc)] = v[q];
            }
        }
    }
}

// z plane k: stage b (or D v / D W^-1 v from the faces, DIV = 1 / 2), x and
// y forward transforms; Y[k][y mode][x mode]
template <typename Tc, int DIV>
__global__ __launch_bounds__(PNT) void k_plane_fwd(PlaneAxes<Tc> a, const double *__restrict__ X,
                                                   Tc *__restrict__ Y, Geo dg) {
    __shared__ Tc P[PCAP];
    typedef typename Mfma<Tc>::acc acc_t;
    const int k = blockIdx.x;
    const int nx = a.n[0], ny = a.n[1], LD = nx + 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (DIV) {
        stage_plane<4>(P, LD, ny, nx, tid, [&](int j, int i) {
            double f[6];
            tpf::cell_faces(dg, X, i + 1, j + 1, k + 1, f);
            return Tc(tpf::cell_div<DIV ? DIV : 1>(dg, f, i + 1, j + 1, k + 1));
        });
    } else {
        const double *src = X + long(k) * nx * ny;
        stage_plane<16>(P, LD, ny, nx, tid, [&](int j, int i) { return Tc(src[j * nx + i]); });
    }
    lds_barrier();
    fold_rows(P, LD, nx, ny, tid);
    lds_barrier();
    acc_t ae[UMAX], ao[UMAX];
    Units u = units_of(nx, ny, wv);
    plane_transform<Tc, true, true>(P, LD, nx, ny, a.fwd[0], u, lane, ae, ao);
    lds_barrier();   // every wave has read the plane
    {
        const int nex = nx - nx / 2, nox = nx / 2;
        const int t = u.tb + (lane & 15);
#pragma unroll
        for (int q = 0; q < UMAX; ++q) {
            if (q >= u.nu) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = (u.pt0 + q * u.dpt) * 16 + Mfma<Tc>::row(lane, r);
                if (p >= ny) continue;
                if (t < nex) P[p * LD + t] = ae[q][r];
                if (t < nox) P[p * LD + nex + t] = ao[q][r];
            }
        }
    }
    lds_barrier();
    fold_cols(P, LD, ny, nx, tid);
    lds_barrier();
    u = units_of(ny, nx, wv);
    plane_transform<Tc, false, true>(P, LD, ny, nx, a.fwd[1], u, lane, ae, ao);
    const int ney = ny - ny / 2, noy = ny / 2;
    Tc *dst = Y + long(k) * nx * ny;
#pragma unroll
    for (int q = 0; q < UMAX; ++q) {
        if (q >= u.nu) continue;
        const int p = (u.pt0 + q * u.dpt) * 16 + (lane & 15);
        if (p >= nx) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = u.tb + Mfma<Tc>::row(lane, r);
            if (t < ney) dst[t * nx + p] = ae[q][r];
            if (t < noy) dst[(ney + t) * nx + p] = ao[q][r];
        }
    }
}

// y plane j: z forward transform, scaling, z inverse transform (in x and y
// modes throughout); Y[k][j][x mode]
template <typename Tc>
__global__ __launch_bounds__(PNT) void k_plane_mid(PlaneAxes<Tc> a, const Tc *__restrict__ X,
                                                   Tc *__restrict__ Y, const Tc *__restrict__ lamy) {
    __shared__ Tc P[PCAP];
    typedef typename Mfma<Tc>::acc acc_t;
    const int j = blockIdx.x;
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2], LD = nx + 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long pl = long(nx) * ny;
    const int ne = nz - nz / 2, no = nz / 2;
    const Units u = units_of(nz, nx, wv);
    // the z eigenvalues and the x eigenvalues + this plane's y eigenvalue,
    // staged with the plane (registers are short here)
    __shared__ Tc L[2 * PMAX];
    {
        const Tc ly = lamy[j];
        for (int e = tid; e < nz; e += PNT) L[e] = a.lam[2][e];
        for (int e = tid; e < nx; e += PNT) L[PMAX + e] = a.lam[0][e] + ly;
    }
    stage_plane<16>(P, LD, nz, nx, tid,
                    [&](int kk, int i) { return X[kk * pl + long(j) * nx + i]; });
    lds_barrier();
    fold_cols(P, LD, nz, nx, tid);
    lds_barrier();
    acc_t ae[UMAX], ao[UMAX];
    plane_transform<Tc, false, true>(P, LD, nz, nx, a.fwd[2], u, lane, ae, ao);
    lds_barrier();   // every wave has read the plane
#pragma unroll
    for (int q = 0; q < UMAX; ++q) {
        if (q >= u.nu) continue;
        const int p = (u.pt0 + q * u.dpt) * 16 + (lane & 15);
        if (p >= nx) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = u.tb + Mfma<Tc>::row(lane, r);
            // the eigenvalue sum vanishes exactly on the singular
            // (all-constant) mode: mapped to 0
            if (t < ne) {
                const Tc den = L[t] + L[PMAX + p];
                P[t * LD + p] = den == Tc(0) ? Tc(0) : ae[q][r] * recip(den);
            }
            if (t < no) {
                const Tc den = L[ne + t] + L[PMAX + p];
                P[(ne + t) * LD + p] = den == Tc(0) ? Tc(0) : ao[q][r] * recip(den);
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);   // no hoisting of the next factors over the scaling
    lds_barrier();
    plane_transform<Tc, false, false>(P, LD, nz, nx, a.inv[2], u, lane, ae, ao);
#pragma unroll
    for (int q = 0; q < UMAX; ++q) {
        if (q >= u.nu) continue;
        const int p = (u.pt0 + q * u.dpt) * 16 + (lane & 15);
        if (p >= nx) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = u.tb + Mfma<Tc>::row(lane, r);
            if (t < no) {
                Y[t * pl + long(j) * nx + p] = ae[q][r] + ao[q][r];
                Y[(nz - 1 - t) * pl + long(j) * nx + p] = ae[q][r] - ao[q][r];
            } else if (t < ne) {
                Y[t * pl + long(j) * nx + p] = ae[q][r];   // the middle (odd N)
            }
        }
    }
}

// z plane k: y inverse and x inverse transforms; phi[k][j][i]
template <typename Tc>
__global__ __launch_bounds__(PNT) void k_plane_inv(PlaneAxes<Tc> a, const Tc *__restrict__ X,
                                                   double *__restrict__ phi) {
    __shared__ Tc P[PCAP];
    typedef typename Mfma<Tc>::acc acc_t;
    const int k = blockIdx.x;
    const int nx = a.n[0], ny = a.n[1], LD = nx + 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const Tc *src = X + long(k) * nx * ny;
    stage_plane<16>(P, LD, ny, nx, tid, [&](int j, int i) { return src[j * nx + i]; });
    lds_barrier();
    acc_t ae[UMAX], ao[UMAX];
    Units u = units_of(ny, nx, wv);
    plane_transform<Tc, false, false>(P, LD, ny, nx, a.inv[1], u, lane, ae, ao);
    lds_barrier();   // every wave has read the plane
    {
        const int ne = ny - ny / 2, no = ny / 2;
#pragma unroll
        for (int q = 0; q < UMAX; ++q) {
            if (q >= u.nu) continue;
            const int p = (u.pt0 + q * u.dpt) * 16 + (lane & 15);
            if (p >= nx) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = u.tb + Mfma<Tc>::row(lane, r);
                if (t < no) {
                    P[t * LD + p] = ae[q][r] + ao[q][r];
                    P[(ny - 1 - t) * LD + p] = ae[q][r] - ao[q][r];
                } else if (t < ne) {
                    P[t * LD + p] = ae[q][r];
                }
            }
        }
    }
    lds_barrier();
    u = units_of(nx, ny, wv);
    plane_transform<Tc, true, false>(P, LD, nx, ny, a.inv[0], u, lane, ae, ao);
    const int ne = nx - nx / 2, no = nx / 2;
    const int t = u.tb + (lane & 15);
    double *dst = phi + long(k) * nx * ny;
#pragma unroll
    for (int q = 0; q < UMAX; ++q) {
        if (q >= u.nu) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = (u.pt0 + q * u.dpt) * 16 + Mfma<Tc>::row(lane, r);
            if (p >= ny) continue;
            if (t < no) {
                dst[p * nx + t] = double(ae[q][r] + ao[q][r]);
                dst[p * nx + nx - 1 - t] = double(ae[q][r] - ao[q][r]);
            } else if (t < ne) {
                dst[p * nx + t] = double(ae[q][r]);
            }
        }
    }
}

// one event pair around the forward plane kernel when it forms the
// divergence (the divergence stage), one around the rest (the transforms)
template <typename Tc>
void plane_typed(fvk_ctx *ctx, const PlaneAxes<Tc> &a, const double *b, double *phi, Tc *t0,
                 Tc *t1, const double *vel, int win, hipStream_t st) {
    const Geo &dg = ctx->geo;
    if (vel) {
        timing_begin(ctx, FVK_STAGE_DIV);
        if (win)
            k_plane_fwd<Tc, 2><<<a.n[2], PNT, 0, st>>>(a, vel, t0, dg);
        else
            k_plane_fwd<Tc, 1><<<a.n[2], PNT, 0, st>>>(a, vel, t0, dg);
        timing_end(ctx, FVK_STAGE_DIV);
        timing_begin(ctx, FVK_STAGE_TRANSFORM);
    } else {
        timing_begin(ctx, FVK_STAGE_TRANSFORM);
        k_plane_fwd<Tc, 0><<<a.n[2], PNT, 0, st>>>(a, b, t0, dg);
    }
    k_plane_mid<Tc><<<a.n[1], PNT, 0, st>>>(a, t0, t1, a.lam[1]);
    k_plane_inv<Tc><<<a.n[2], PNT, 0, st>>>(a, t1, phi);
    timing_end(ctx, FVK_STAGE_TRANSFORM, vel ? 2 : 3);
}

}  // namespace

bool tpf_plane_fits(const int n[3]) {
    for (int q = 0; q < 3; ++q)
        if (n[q] < 4 || n[q] > PMAX) return false;
    return true;
}

void tpf_solve_planes(fvk_ctx *ctx, const double *b, double *phi, bool fp32, hipStream_t st,
                      const double *vel, int win) {
    const Workspace &w = ctx->ws;
    if (fp32) {
        PlaneAxes<float> a;
        for (int q = 0; q < 3; ++q) {
            a.fwd[q] = w.Ah32[q];
            a.inv[q] = w.Bh32[q];
            a.lam[q] = w.lamp32[q];
            a.n[q] = ctx->n[q];
        }
        plane_typed<float>(ctx, a, b, phi, static_cast<float *>(w.tb0),
                           static_cast<float *>(w.tb1), vel, win, st);
    } else {
        PlaneAxes<double> a;
        for (int q = 0; q < 3; ++q) {
            a.fwd[q] = w.Ah[q];
            a.inv[q] = w.Bh[q];
            a.lam[q] = w.lamp[q];
            a.n[q] = ctx->n[q];
        }
        plane_typed<double>(ctx, a, b, phi, static_cast<double *>(w.tb0),
                            static_cast<double *>(w.tb1), vel, win, st);
    }
}

}  // namespace fvk
