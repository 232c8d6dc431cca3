// Vector kernels around the Krylov vector: Gram-Schmidt dot products and
// updates (Arnoldi / GMRES orthogonalisation), Krylov-Schur basis rotation,
// reductions.  All reductions use a fixed tree (wavefront shuffles, then the
// block, then a separate pass over the block partials in index order), so
// results are bitwise reproducible run to run.
#include <algorithm>

#include "fvk_internal.h"

namespace fvk {

namespace {

constexpr int NT = 256;
constexpr int GROUP = 16;  // vectors per pass of the multi-dot kernel

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// partials[blk * m + q] = sum over this block's rows of V_q[r] * w[r]
__global__ __launch_bounds__(NT) void k_multidot(const double *__restrict__ V, size_t ldv, int m,
                                                 const double *__restrict__ w, size_t n,
                                                 size_t chunk, double *__restrict__ partials) {
    __shared__ double sh[GROUP][NT / 64];
    const size_t r0 = size_t(blockIdx.x) * chunk;
    const size_t r1 = min(n, r0 + chunk);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q0 = 0; q0 < m; q0 += GROUP) {
        double acc[GROUP];
#pragma unroll
        for (int t = 0; t < GROUP; ++t) acc[t] = 0.0;
        for (size_t r = r0 + threadIdx.x; r < r1; r += NT) {
            const double wr = w[r];
#pragma unroll
            for (int t = 0; t < GROUP; ++t)
                if (q0 + t < m) acc[t] += V[size_t(q0 + t) * ldv + r] * wr;
        }
#pragma unroll
        for (int t = 0; t < GROUP; ++t) {
            const double s = wave_sum(acc[t]);
            if (lane == 0) sh[t][wv] = s;
        }
        __syncthreads();
        if (threadIdx.x < GROUP && q0 + threadIdx.x < m) {
            double s = 0.0;
            for (int q = 0; q < NT / 64; ++q) s += sh[threadIdx.x][q];
            partials[size_t(blockIdx.x) * m + q0 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

// Dot products of m rows of V with two vectors x and y in one pass over V.
// Block b owns the contiguous tile [b T2, (b+1) T2) of the entries (the
// whole chip streams neighbouring tiles, as the update kernel does) and walks
// its rows in groups of GROUP2, re-reading the tile of x and y from L2:
// partials[(2q + r) * nblk + b] = sum over the tile of V_q[i] * (r ? y : x)[i].
constexpr int GROUP2 = 8, E2 = 16, U2 = 4, T2 = NT * E2;
__global__ __launch_bounds__(NT) void k_multidot2(const double *__restrict__ V, size_t ldv, int m,
                                                  const double *__restrict__ x,
                                                  const double *__restrict__ y, size_t n,
                                                  size_t tile, int nblk,
                                                  double *__restrict__ partials) {
    __shared__ double sh[2 * GROUP2][NT / 64];
    const size_t r0 = size_t(blockIdx.x) * tile;
    const size_t r1 = min(n, r0 + tile);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q0 = 0; q0 < m; q0 += GROUP2) {
        double ax[GROUP2], ay[GROUP2];
#pragma unroll
        for (int t = 0; t < GROUP2; ++t) ax[t] = ay[t] = 0.0;
        // U2 entries per step, loads issued together (clamped addresses; the
        // entries past the tile get zero weights)
        for (size_t rb = r0; rb < r1; rb += size_t(U2) * NT) {
            double xr[U2], yr[U2], v[U2][GROUP2];
#pragma unroll
            for (int u = 0; u < U2; ++u) {
                const size_t r = rb + size_t(u) * NT + threadIdx.x;
                const size_t rc = min(r, r1 - 1);
                const bool in = r < r1;
                xr[u] = in ? x[rc] : 0.0;
                yr[u] = in ? y[rc] : 0.0;
#pragma unroll
                for (int t = 0; t < GROUP2; ++t)
                    v[u][t] = V[size_t(min(q0 + t, m - 1)) * ldv + rc];
            }
#pragma unroll
            for (int u = 0; u < U2; ++u)
#pragma unroll
                for (int t = 0; t < GROUP2; ++t) {
                    ax[t] += v[u][t] * xr[u];
                    ay[t] += v[u][t] * yr[u];
                }
        }
#pragma unroll
        for (int t = 0; t < GROUP2; ++t) {
            const double sx = wave_sum(ax[t]), sy = wave_sum(ay[t]);
            if (lane == 0) {
                sh[2 * t][wv] = sx;
                sh[2 * t + 1][wv] = sy;
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * GROUP2 && q0 + threadIdx.x / 2 < m) {
            double s = 0.0;
            for (int q = 0; q < NT / 64; ++q) s += sh[threadIdx.x][q];
            partials[size_t(2 * q0 + threadIdx.x) * nblk + blockIdx.x] = s;
        }
        __syncthreads();
    }
}

// out[q] = sum_b partials[q * nblk + b] (rows of block partials, contiguous)
__global__ void k_reduce_rows(const double *__restrict__ partials, int nblk,
                              double *__restrict__ out) {
    const int q = blockIdx.x;
    __shared__ double sh[NT / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NT) s += partials[size_t(q) * nblk + b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NT / 64; ++k) t += sh[k];
        out[q] = t;
    }
}

// The two updates of the lagged CGS2 step in one pass over V_0..V_{m-1}:
// x <- c1 x + sum_q a[q] V_q and y <- c2 y + c3 x_old + sum_q b[q] V_q
// (a, b on the device; x, y distinct from the V_q).
__global__ __launch_bounds__(NT) void k_update2(double *__restrict__ x, double *__restrict__ y,
                                                const double *__restrict__ V, size_t ldv, int m,
                                                const double *__restrict__ a,
                                                const double *__restrict__ b, double c1,
                                                double c2, double c3, size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r >= n) return;
    double sa = 0.0, sb = 0.0;
#pragma unroll 8
    for (int q = 0; q < m; ++q) {
        const double v = V[size_t(q) * ldv + r];
        sa += a[q] * v;
        sb += b[q] * v;
    }
    const double xo = x[r];
    x[r] = c1 * xo + sa;
    y[r] = c2 * y[r] + c3 * xo + sb;
}

// out[q] = (accumulate ? out[q] : 0) + sum_blk partials[blk * m + q]
__global__ void k_reduce_partials(const double *__restrict__ partials, int nblk, int m,
                                  double *__restrict__ out, int accumulate) {
    const int q = blockIdx.x;
    __shared__ double sh[NT / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NT) s += partials[size_t(b) * m + q];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NT / 64; ++k) t += sh[k];
        out[q] = accumulate ? out[q] + t : t;
    }
}

// w = alpha w + beta sum_q c[q] V_q   (c on the device)
__global__ __launch_bounds__(NT) void k_multiaxpy(double *__restrict__ w, double alpha,
                                                  double beta, const double *__restrict__ V,
                                                  size_t ldv, int m, const double *__restrict__ c,
                                                  size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r >= n) return;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < m; ++q) s += c[q] * V[size_t(q) * ldv + r];
    w[r] = alpha * w[r] + beta * s;
}

// V[:, p] = sum_q V[:, q] Q[q + p*m] for p < k, rows staged in LDS.
constexpr int ROT_ROWS = 32;
__global__ __launch_bounds__(NT) void k_basis_rotate(double *__restrict__ V, size_t ldv, int m,
                                                     const double *__restrict__ Q, int k,
                                                     size_t n) {
    extern __shared__ double sv[];   // ROT_ROWS * m
    const size_t r0 = size_t(blockIdx.x) * ROT_ROWS;
    for (int e = threadIdx.x; e < ROT_ROWS * m; e += NT) {
        const int rr = e % ROT_ROWS, q = e / ROT_ROWS;
        const size_t r = r0 + rr;
        sv[q * ROT_ROWS + rr] = (r < n) ? V[size_t(q) * ldv + r] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ROT_ROWS * k; e += NT) {
        const int rr = e % ROT_ROWS, p = e / ROT_ROWS;
        const size_t r = r0 + rr;
        if (r >= n) continue;
        double s = 0.0;
        for (int q = 0; q < m; ++q) s += sv[q * ROT_ROWS + rr] * Q[size_t(p) * m + q];
        V[size_t(p) * ldv + r] = s;
    }
}

// slots: out[0] = max of partials; running[0] = max(running, out);
// count_over[0] += (out >= tol).  One block of 1024 threads; each thread
// issues its loads back to back (independent) before reducing.
constexpr int NTR = 1024;
__global__ __launch_bounds__(NTR) void k_max_reduce(const double *__restrict__ partials, int nblk,
                                                    double *out, double *running,
                                                    int *count_over, double tol) {
    __shared__ double sh[NTR / 64];
    double v = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * NTR < nblk; b += 4 * NTR) {
        const double a0 = partials[b], a1 = partials[b + NTR], a2 = partials[b + 2 * NTR],
                     a3 = partials[b + 3 * NTR];
        v = fmax(v, fmax(fmax(a0, a1), fmax(a2, a3)));
    }
    for (; b < nblk; b += NTR) v = fmax(v, partials[b]);
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NTR / 64; ++k) t = fmax(t, sh[k]);
        out[0] = t;
        if (running) running[0] = fmax(running[0], t);
        if (count_over && !(t < tol)) count_over[0] += 1;
    }
}

// the asynchronous divergence records: row e holds the block maxima of one
// call; one block reduces the rows in call order
__global__ __launch_bounds__(NTR) void k_ring_reduce(const double *__restrict__ rows, int nblk,
                                                     int n, double *running, int *count_over,
                                                     double tol) {
    __shared__ double sh[NTR / 64];
    double run = 0.0;
    int cnt = 0;
    for (int e = 0; e < n; ++e) {
        const double *r = rows + long(e) * nblk;
        double v = 0.0;
        for (int b = threadIdx.x; b < nblk; b += NTR) v = fmax(v, r[b]);
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int k = 0; k < NTR / 64; ++k) t = fmax(t, sh[k]);
            run = fmax(run, t);
            if (!(t < tol)) ++cnt;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        running[0] = fmax(running[0], run);
        count_over[0] += cnt;
    }
}

// partials[blk] = max |x| over the block's rows
__global__ __launch_bounds__(NT) void k_absmax(const double *__restrict__ x, size_t n,
                                               size_t chunk, double *__restrict__ partials) {
    __shared__ double sh[NT / 64];
    const size_t r0 = size_t(blockIdx.x) * chunk;
    const size_t r1 = min(n, r0 + chunk);
    double v = 0.0;
    for (size_t r = r0 + threadIdx.x; r < r1; r += NT) v = fmax(v, fabs(x[r]));
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NT / 64; ++k) t = fmax(t, sh[k]);
        partials[blockIdx.x] = t;
    }
}

__global__ void k_scale_by_inv_sqrt(double *__restrict__ w, const double *__restrict__ nrm2,
                                    size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r >= n) return;
    const double s = nrm2[0];
    if (s > 0.0) w[r] *= 1.0 / sqrt(s);
}

__global__ void k_axpby(double *__restrict__ y, double a, const double *__restrict__ x, double b,
                        size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r >= n) return;
    y[r] = a * x[r] + b * y[r];
}

__global__ void k_lincomb3(double *__restrict__ z, double a, const double *__restrict__ x,
                           double b, const double *__restrict__ y, double c, size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r >= n) return;
    z[r] = a * x[r] + b * y[r] + c * z[r];
}

__global__ void k_fill(double *__restrict__ y, double v, size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r < n) y[r] = v;
}

__global__ void k_copy(double *__restrict__ y, const double *__restrict__ x, size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r < n) y[r] = x[r];
}

__global__ void k_scale(double *__restrict__ y, double a, size_t n) {
    const size_t r = size_t(blockIdx.x) * NT + threadIdx.x;
    if (r < n) y[r] *= a;
}

inline unsigned nblk1(size_t n) { return unsigned((n + NT - 1) / NT); }

}  // namespace

int multidot_blocks(size_t n) {
    size_t b = (n + 4095) / 4096;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return int(b);
}

void launch_multidot(const double *V, size_t ldv, int m, const double *w, size_t n,
                     double *partials, int nblk, hipStream_t st) {
    const size_t chunk = (n + nblk - 1) / nblk;
    k_multidot<<<nblk, NT, 0, st>>>(V, ldv, m, w, n, chunk, partials);
}

// One resident round of the two-vector dot kernel (three 256-thread blocks per
// compute unit at its register count, 256 compute units): a second, partial
// round would leave most of the chip idle.
// tiles of T2 entries, at most 32768 of them (longer tiles beyond that)
int multidot2_blocks(size_t n) {
    const size_t b = (n + T2 - 1) / T2;
    return int(std::max<size_t>(1, std::min<size_t>(b, 32768)));
}

// partials: 2 m rows of nblk block sums; out: the 2 m dot products
// (out[2q] = V_q . x, out[2q + 1] = V_q . y)
void launch_multidot2(const double *V, size_t ldv, int m, const double *x, const double *y,
                      size_t n, double *partials, int nblk, double *out, hipStream_t st) {
    const size_t tile = (n + nblk - 1) / nblk;
    k_multidot2<<<nblk, NT, 0, st>>>(V, ldv, m, x, y, n, tile, nblk, partials);
    k_reduce_rows<<<2 * m, NT, 0, st>>>(partials, nblk, out);
}

void launch_update2(double *x, double *y, const double *V, size_t ldv, int m, const double *a_dev,
                    const double *b_dev, double c1, double c2, double c3, size_t n,
                    hipStream_t st) {
    k_update2<<<nblk1(n), NT, 0, st>>>(x, y, V, ldv, m, a_dev, b_dev, c1, c2, c3, n);
}

void launch_reduce_partials(const double *partials, int nblk, int m, double *out, int accumulate,
                            hipStream_t st) {
    k_reduce_partials<<<m, NT, 0, st>>>(partials, nblk, m, out, accumulate);
}

void launch_multiaxpy(double *w, double alpha, double beta, const double *V, size_t ldv, int m,
                      const double *c_dev, size_t n, hipStream_t st) {
    k_multiaxpy<<<nblk1(n), NT, 0, st>>>(w, alpha, beta, V, ldv, m, c_dev, n);
}

void launch_basis_rotate(double *V, size_t ldv, int m, const double *Q_dev, int k, size_t n,
                         hipStream_t st) {
    const unsigned nb = unsigned((n + ROT_ROWS - 1) / ROT_ROWS);
    k_basis_rotate<<<nb, NT, size_t(ROT_ROWS) * m * sizeof(double), st>>>(V, ldv, m, Q_dev, k, n);
}

void launch_max_reduce(const double *partials, int nblk, double *out, double *running,
                       int *count_over, double tol, hipStream_t st) {
    k_max_reduce<<<1, NTR, 0, st>>>(partials, nblk, out, running, count_over, tol);
}

void launch_ring_reduce(const double *rows, int nblk, int n, double *running, int *count_over,
                        double tol, hipStream_t st) {
    k_ring_reduce<<<1, NTR, 0, st>>>(rows, nblk, n, running, count_over, tol);
}

void launch_absmax(const double *x, size_t n, double *partials, int nblk, hipStream_t st) {
    const size_t chunk = (n + nblk - 1) / nblk;
    k_absmax<<<nblk, NT, 0, st>>>(x, n, chunk, partials);
}

void launch_scale_inv_sqrt(double *w, const double *nrm2, size_t n, hipStream_t st) {
    k_scale_by_inv_sqrt<<<nblk1(n), NT, 0, st>>>(w, nrm2, n);
}

void launch_axpby(double *y, double a, const double *x, double b, size_t n, hipStream_t st) {
    k_axpby<<<nblk1(n), NT, 0, st>>>(y, a, x, b, n);
}

void launch_lincomb3(double *z, double a, const double *x, double b, const double *y, double c,
                     size_t n, hipStream_t st) {
    k_lincomb3<<<nblk1(n), NT, 0, st>>>(z, a, x, b, y, c, n);
}

void launch_fill(double *y, double v, size_t n, hipStream_t st) {
    k_fill<<<nblk1(n), NT, 0, st>>>(y, v, n);
}

void launch_copy(double *dst, const double *src, size_t n, hipStream_t st) {
    k_copy<<<nblk1(n), NT, 0, st>>>(dst, src, n);
}

void launch_scale(double *w, double alpha, size_t n, hipStream_t st) {
    k_scale<<<nblk1(n), NT, 0, st>>>(w, alpha, n);
}

}  // namespace fvk
