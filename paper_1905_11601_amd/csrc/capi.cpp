// C-ABI entry points of the fvk library: context management, the operators of
// the Krylov-vector path (paper Sec. 3.1) and the Arnoldi step around them.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "fvk_internal.h"

using namespace fvk;

#define HIPCHK(ctx, call)                                                              \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
            return FVK_EHIP;                                                           \
        }                                                                              \
    } while (0)

#define CHECK_LAUNCH(ctx) HIPCHK(ctx, hipGetLastError())

namespace {

fvk_status fail(fvk_ctx *ctx, fvk_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

template <typename T>
fvk_status dalloc(fvk_ctx *ctx, T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) {
        ctx->err = std::string("hipMalloc: ") + hipGetErrorString(e);
        *p = nullptr;
        return FVK_ENOMEM;
    }
    return FVK_OK;
}

void free_ws(fvk_ctx *ctx) {
    Workspace &w = ctx->ws;
    auto fr = [](void *p) {
        if (p) (void)hipFree(p);
    };
    fr(w.geo);
    fr(w.div);
    fr(w.phi);
    fr(w.tb0);
    fr(w.tb1);
    for (int a = 0; a < 3; ++a) {
        fr(w.E[a]);
        fr(w.Einv[a]);
        fr(w.lam[a]);
        fr(w.E32[a]);
        fr(w.Einv32[a]);
        fr(w.lam32[a]);
        fr(w.Ah[a]);
        fr(w.Bh[a]);
        fr(w.lamp[a]);
        fr(w.Ah32[a]);
        fr(w.Bh32[a]);
        fr(w.lamp32[a]);
    }
    fr(w.vtmp);
    fr(w.vtmp2);
    fr(w.red);
    fr(w.dev_scalars);
    fr(w.ring);
    fr(w.dev_counters);
    fr(w.div_slots);
    fr(w.coef_dev);
    fr(w.zeros);
    if (w.host_pinned) (void)hipHostFree(w.host_pinned);
    w = Workspace();
}

void set_coefs_from_params(fvk_ctx *ctx) {
    ctx->co.nu = 1.0 / std::sqrt(ctx->Gr);
    ctx->co.kappa = ctx->co.nu / ctx->Pr;
    ctx->co.b = 1.0;
}

size_t nvec(const fvk_ctx *ctx) { return size_t(4) * size_t(ctx->geo.F); }

// Read `count` doubles from device memory into host `out` (synchronises).
fvk_status read_back(fvk_ctx *ctx, const double *dev, double *out, size_t count) {
    if (count > ctx->ws.host_pinned_len) return fail(ctx, FVK_EINVAL, "read_back too large");
    HIPCHK(ctx, hipMemcpyAsync(ctx->ws.host_pinned, dev, count * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(out, ctx->ws.host_pinned, count * sizeof(double));
    return FVK_OK;
}

fvk_status write_coefs(fvk_ctx *ctx, const double *host, size_t count) {
    if (count > ctx->ws.coef_len) return fail(ctx, FVK_EINVAL, "too many coefficients");
    // stage through pinned memory so the copy is stream-ordered
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(ctx->ws.host_pinned, host, count * sizeof(double));
    HIPCHK(ctx, hipMemcpyAsync(ctx->ws.coef_dev, ctx->ws.host_pinned, count * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return FVK_OK;
}

// Reduce the pending asynchronous divergence records into the running maximum
// and the count of calls above tolerance (stream-ordered after the calls).
void flush_ring(fvk_ctx *ctx) {
    Workspace &w = ctx->ws;
    if (w.ring_n == 0) return;
    launch_ring_reduce(w.ring, correct_blocks(ctx->geo), w.ring_n, w.div_slots + 1,
                       w.dev_counters, ctx->simple_tol, ctx->stream);
    w.ring_n = 0;
}

// ---- SIMPLE loop (Sec. 3.1, steps 1-3) ------------------------------------
// vin: 3 velocity fields (the momentum predictor; its wall entries are not
// read); vout: result (3 fields); spare: a third 3-field buffer for the
// ping-pong of later passes (it may be vin when vin may be clobbered; it must
// differ from vout).  sync: adaptive loop with a host check per pass;
// otherwise a fixed number of passes and the divergence test is recorded on
// the device.  transposed: the transposed projection W P W^-1 (P is
// W-orthogonal, W = face control volumes): the first pass reads W^-1 vin and
// the result is scaled by W, fused into the kernels where the pass count is
// known in advance.
fvk_status simple_forward(fvk_ctx *ctx, const double *vin, double *vout, double *spare,
                          double *p_out, bool sync, int *passes_out, double *div_out,
                          bool transposed = false) {
    const Geo &g = ctx->geo;
    Workspace &w = ctx->ws;
    hipStream_t st = ctx->stream;
    const bool fp32 = ctx->prec == FVK_MIXED;
    const int fixed = fp32 ? ctx->mixed_passes : 1;
    // the transposed loop always runs the fixed pass count: its divergence is
    // that of the internal field W^-1 y, whose size (and rounding floor) has
    // no relation to the absolute tolerance of the physical velocity;
    // passes/div are still reported
    bool want_div = sync;
    if (transposed) sync = false;
    // the number of FP32 solves + FP64 refinement passes that reach the
    // tolerance depends on the grid and the operator's scale (2 at 100^3, 3
    // at 256^3): the first asynchronous forward call in mixed precision runs
    // the adaptive loop and fixes the count of the later asynchronous ones
    const bool calibrate = fp32 && !sync && !transposed && !ctx->mixed_calibrated;
    if (calibrate) sync = want_div = true;
    if (p_out) launch_fill(p_out, 0.0, ctx->ncell, st);
    // first right-hand side D vin: formed inside the first transform where the
    // x axis allows it, else by the divergence kernel
    const bool fused_div = tpf_fuses_div(ctx);
    if (!fused_div) {
        timing_begin(ctx, FVK_STAGE_DIV);
        launch_div(g, vin, w.div, st, transposed);
        timing_end(ctx, FVK_STAGE_DIV);
    }
    const double *src = vin;
    double *dst = vout, *other = spare;
    int k = 0;
    double dmax = 0.0;
    bool scaled_out = false;
    while (true) {
        if (k == 0 && fused_div)
            tpf_solve(ctx, nullptr, w.phi, fp32, st, vin, transposed ? 1 : 0);
        else
            tpf_solve(ctx, w.div, w.phi, fp32, st);
        const bool last_fixed = !sync && k + 1 >= fixed;
        const bool win = transposed && k == 0, wout = transposed && last_fixed;
        timing_begin(ctx, FVK_STAGE_CORRECT);
        // D v of the result is the next pass's right-hand side; after the last
        // pass of a fixed count only its maximum (the block maxima) is needed.
        // The running record of asynchronous calls covers forward projections:
        // their block maxima go to the next row of the ring, reduced kRing
        // calls at a time (no reduction launch per call); other passes reduce
        // at once
        const bool record = last_fixed && !transposed;
        if (record) {
            launch_correct_oop(g, src, dst, w.phi, p_out, nullptr,
                               w.ring + size_t(w.ring_n) * correct_blocks(g), st, win, wout);
            if (++w.ring_n == kRing) flush_ring(ctx);
        } else {
            launch_correct_oop(g, src, dst, w.phi, p_out, last_fixed ? nullptr : w.div, w.red,
                               st, win, wout);
            launch_max_reduce(w.red, correct_blocks(g), w.div_slots, nullptr, nullptr,
                              ctx->simple_tol, st);
        }
        timing_end(ctx, FVK_STAGE_CORRECT);
        CHECK_LAUNCH(ctx);
        scaled_out = wout;
        if (sync) {
            fvk_status s = read_back(ctx, w.div_slots, &dmax, 1);
            if (s != FVK_OK) return s;
        }
        ++k;
        if (sync) {
            if (dmax < ctx->simple_tol || k >= ctx->simple_cap) break;
        } else if (k >= fixed) {
            break;
        }
        src = dst;
        std::swap(dst, other);
    }
    if (dst != vout) launch_copy(vout, dst, size_t(3) * g.F, st);
    if (transposed && !scaled_out) launch_face_scale(g, vout, vout, 0, st);
    CHECK_LAUNCH(ctx);
    if (want_div && !sync) {
        fvk_status s = read_back(ctx, w.div_slots, &dmax, 1);
        if (s != FVK_OK) return s;
    }
    if (passes_out) *passes_out = k;
    if (div_out) *div_out = dmax;
    if (sync && !(dmax < ctx->simple_tol))
        return fail(ctx, FVK_ENOCONV, "SIMPLE loop hit its pass cap");
    if (calibrate) {
        // vectors differ by a factor ~2 in the divergence a given pass count
        // leaves (each pass contracts it ~1e-6-fold): a result within 10x of
        // the tolerance means another vector may miss it, so one pass more
        ctx->mixed_passes = std::max(2, dmax > 0.1 * ctx->simple_tol ? k + 1 : k);
        ctx->mixed_calibrated = true;
    }
    return FVK_OK;
}

// Transposed SIMPLE projection of a velocity part: z = P^T y = W P W^-1 y,
// i.e. the forward loop -- including its FP32 solves with FP64 refinement in
// mixed mode -- between two diagonal scalings, fused into its first and last
// pass.  y is not modified; z may be any 3-field buffer except ws.vtmp2.
fvk_status simple_transpose(fvk_ctx *ctx, const double *y, double *z, bool sync,
                            int *passes_out, double *div_out) {
    return simple_forward(ctx, y, z, ctx->ws.vtmp2, nullptr, sync, passes_out, div_out, true);
}

}  // namespace

namespace fvk {

static constexpr size_t kTimingPairs = 8192;

static void timing_harvest(fvk_ctx *ctx) {
    Timing &t = ctx->tm;
    if (t.used == 0) return;
    (void)hipEventSynchronize(t.ev[2 * (t.used - 1) + 1]);
    for (size_t q = 0; q < t.used; ++q) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.ev[2 * q], t.ev[2 * q + 1]) == hipSuccess) {
            t.ms[t.stage[q]] += ms;
            t.count[t.stage[q]] += t.launches[q];
        }
    }
    t.used = 0;
}

void timing_begin(fvk_ctx *ctx, int stage) {
    Timing &t = ctx->tm;
    if (!(t.mask & (1 << stage))) return;
    if (t.used == kTimingPairs) timing_harvest(ctx);
    (void)hipEventRecord(t.ev[2 * t.used], ctx->stream);
    t.stage[t.used] = stage;
}

void timing_end(fvk_ctx *ctx, int stage, int launches) {
    Timing &t = ctx->tm;
    if (!(t.mask & (1 << stage))) return;
    (void)hipEventRecord(t.ev[2 * t.used + 1], ctx->stream);
    t.launches[t.used] = launches;
    ++t.used;
}

}  // namespace fvk

extern "C" {

fvk_status fvk_set_timing(fvk_ctx *ctx, int mask) {
    if (!ctx || mask < 0 || mask >= (1 << FVK_NSTAGES)) return FVK_EINVAL;
    Timing &t = ctx->tm;
    if (mask && t.ev.empty()) {
        t.ev.resize(2 * kTimingPairs);
        t.stage.resize(kTimingPairs);
        t.launches.resize(kTimingPairs);
        for (auto &e : t.ev) HIPCHK(ctx, hipEventCreate(&e));
    }
    timing_harvest(ctx);
    t.mask = mask;
    return FVK_OK;
}

fvk_status fvk_timing_read(fvk_ctx *ctx, double *ms, int *counts) {
    if (!ctx) return FVK_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    timing_harvest(ctx);
    Timing &t = ctx->tm;
    for (int s = 0; s < FVK_NSTAGES; ++s) {
        if (ms) ms[s] = t.ms[s];
        if (counts) counts[s] = t.count[s];
        t.ms[s] = 0.0;
        t.count[s] = 0;
    }
    return FVK_OK;
}

fvk_status fvk_create(fvk_ctx **out, int nx, int ny, int nz, int grid_kind, double s, int span_bc,
                      double Gr, double Pr, int prec, void *hip_stream) {
    if (!out) return FVK_EINVAL;
    *out = nullptr;
    if (nx < 2 || ny < 2 || nz < 2 || nx > 1024 || ny > 1024 || nz > 1024) return FVK_EINVAL;
    if (grid_kind < 0 || grid_kind > 2 || (span_bc != 0 && span_bc != 1)) return FVK_EINVAL;
    if (prec != FVK_FP64 && prec != FVK_MIXED) return FVK_EINVAL;
    if (!(Gr > 0) || !(Pr > 0)) return FVK_EINVAL;
    if (grid_kind == FVK_GRID_SINE && !(s >= 0 && s < 1.0 / (2.0 * M_PI))) return FVK_EINVAL;
    if (grid_kind == FVK_GRID_TANH && !(s > 0)) return FVK_EINVAL;
    fvk_ctx *ctx = new (std::nothrow) fvk_ctx();
    if (!ctx) return FVK_ENOMEM;
    ctx->n[0] = nx;
    ctx->n[1] = ny;
    ctx->n[2] = nz;
    ctx->kind = grid_kind;
    ctx->s = s;
    ctx->bc = span_bc;
    ctx->Gr = Gr;
    ctx->Pr = Pr;
    ctx->prec = prec;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    set_coefs_from_params(ctx);
    for (int a = 0; a < 3; ++a) {
        build_axis(ctx->ax[a], ctx->n[a], grid_kind, s);
        neumann_eig(ctx->ax[a], ctx->eig[a]);
        if (ctx->n[a] <= kSymMax) neumann_eig_sym(ctx->ax[a], ctx->esym[a]);
    }
    Geo &g = ctx->geo;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = ctx->n[a];
        g.np[a] = ctx->n[a] + 2;
    }
    g.s[0] = 1;
    g.s[1] = g.np[0];
    g.s[2] = long(g.np[0]) * g.np[1];
    g.F = g.s[2] * g.np[2];
    ctx->ncell = size_t(nx) * ny * nz;

    fvk_status st = FVK_OK;
    Workspace &w = ctx->ws;
    // geometry: per axis 3 arrays of n+4 entries (offset by one)
    std::vector<double> geo;
    size_t off[3][3];
    for (int a = 0; a < 3; ++a) {
        const AxisHost &ah = ctx->ax[a];
        const int n = ah.n;
        std::vector<double> ih(n + 4, 0.0), id(n + 4, 0.0), ww(n + 4, 0.0);
        for (int i = 1; i <= n; ++i) ih[i + 1] = 1.0 / ah.h[i];
        for (int i = 0; i <= n; ++i) id[i + 1] = 1.0 / ah.d[i];
        for (int i = 0; i <= n; ++i) ww[i + 1] = ah.w[i];
        off[a][0] = geo.size();
        geo.insert(geo.end(), ih.begin(), ih.end());
        off[a][1] = geo.size();
        geo.insert(geo.end(), id.begin(), id.end());
        off[a][2] = geo.size();
        geo.insert(geo.end(), ww.begin(), ww.end());
    }
    const size_t nc = ctx->ncell;
    if ((st = dalloc(ctx, &w.geo, geo.size())) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.div, nc)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.phi, nc)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, reinterpret_cast<double **>(&w.tb0), nc)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, reinterpret_cast<double **>(&w.tb1), nc)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.vtmp, nvec(ctx))) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.vtmp2, nvec(ctx))) != FVK_OK) goto bad;
    // block partials: multi-dot (<= 1024 vectors) and the lagged step's
    // two-vector dots (2 (j + 2) <= 1024 rows: Krylov dimensions up to 510,
    // beyond the 400 of fvk_linear_solve / newton_step's GMRES(m))
    w.red_len = std::max<size_t>(size_t(correct_blocks(g)),
                                 size_t(std::max(multidot_blocks(nvec(ctx)),
                                                 multidot2_blocks(nvec(ctx)))) * 1024);
    if ((st = dalloc(ctx, &w.red, w.red_len)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.dev_scalars, 4096)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.ring, size_t(kRing) * correct_blocks(g))) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.dev_counters, 16)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.div_slots, 4)) != FVK_OK) goto bad;
    w.coef_len = 65536;
    if ((st = dalloc(ctx, &w.coef_dev, w.coef_len)) != FVK_OK) goto bad;
    if ((st = dalloc(ctx, &w.zeros, size_t(std::max(nx, std::max(ny, nz))))) != FVK_OK) goto bad;
    if (hipMemset(w.zeros, 0, sizeof(double) * size_t(std::max(nx, std::max(ny, nz)))) !=
        hipSuccess) {
        st = fail(ctx, FVK_EHIP, "zeroing failed");
        goto bad;
    }
    w.host_pinned_len = 65536;
    if (hipHostMalloc(reinterpret_cast<void **>(&w.host_pinned),
                      w.host_pinned_len * sizeof(double), 0) != hipSuccess) {
        w.host_pinned = nullptr;
        st = fail(ctx, FVK_ENOMEM, "hipHostMalloc failed");
        goto bad;
    }
    for (int a = 0; a < 3; ++a) {
        const int n = ctx->n[a];
        const Eig1D &e = ctx->eig[a];
        if ((st = dalloc(ctx, &w.E[a], size_t(n) * n)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.Einv[a], size_t(n) * n)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.lam[a], n)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.E32[a], size_t(n) * n)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.Einv32[a], size_t(n) * n)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.lam32[a], n)) != FVK_OK) goto bad;
        std::vector<float> E32(e.E.begin(), e.E.end()), Ei32(e.Einv.begin(), e.Einv.end()),
            l32(e.lam.begin(), e.lam.end());
        if (hipMemcpy(w.E[a], e.E.data(), e.E.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(w.Einv[a], e.Einv.data(), e.Einv.size() * 8, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(w.lam[a], e.lam.data(), e.lam.size() * 8, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(w.E32[a], E32.data(), E32.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(w.Einv32[a], Ei32.data(), Ei32.size() * 4, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(w.lam32[a], l32.data(), l32.size() * 4, hipMemcpyHostToDevice) !=
                hipSuccess) {
            st = fail(ctx, FVK_EHIP, "eigenbasis upload failed");
            goto bad;
        }
    }
    for (int a = 0; a < 3; ++a) {
        if (ctx->n[a] > kSymMax) continue;
        const EigSym &e = ctx->esym[a];
        const size_t ms = e.A.size();
        std::vector<float> A32(e.A.begin(), e.A.end()), B32(e.B.begin(), e.B.end()),
            l32(e.lam.begin(), e.lam.end());
        if ((st = dalloc(ctx, &w.Ah[a], ms)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.Bh[a], ms)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.lamp[a], e.n)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.Ah32[a], ms)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.Bh32[a], ms)) != FVK_OK) goto bad;
        if ((st = dalloc(ctx, &w.lamp32[a], e.n)) != FVK_OK) goto bad;
        if (hipMemcpy(w.Ah[a], e.A.data(), ms * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(w.Bh[a], e.B.data(), ms * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(w.lamp[a], e.lam.data(), e.n * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(w.Ah32[a], A32.data(), ms * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(w.Bh32[a], B32.data(), ms * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(w.lamp32[a], l32.data(), e.n * 4, hipMemcpyHostToDevice) != hipSuccess) {
            st = fail(ctx, FVK_EHIP, "half-size eigenbasis upload failed");
            goto bad;
        }
    }
    if (hipMemcpy(w.geo, geo.data(), geo.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(w.dev_scalars, 0, 4096 * 8) != hipSuccess ||
        hipMemset(w.dev_counters, 0, 16 * sizeof(int)) != hipSuccess ||
        hipMemset(w.div_slots, 0, 4 * sizeof(double)) != hipSuccess) {
        st = fail(ctx, FVK_EHIP, "geometry upload failed");
        goto bad;
    }
    // device address of the non-allocating entry point's static scratch on
    // this device (once per device)
    if (!noalloc_prepare(&ctx->err)) {
        st = FVK_EHIP;
        goto bad;
    }
    for (int a = 0; a < 3; ++a) {
        g.ax[a].ih = w.geo + off[a][0] + 1;
        g.ax[a].id = w.geo + off[a][1] + 1;
        g.ax[a].w = w.geo + off[a][2] + 1;
    }
    *out = ctx;
    return FVK_OK;
bad:
    free_ws(ctx);
    delete ctx;
    return st;
}

fvk_status fvk_destroy(fvk_ctx *ctx) {
    if (!ctx) return FVK_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    free_ws(ctx);
    delete ctx;
    return FVK_OK;
}

fvk_status fvk_set_stream(fvk_ctx *ctx, void *s) {
    if (!ctx) return FVK_EINVAL;
    // every call shares the context's workspace (scratch vectors, Poisson
    // arrays, reduction slots, the record ring): work still queued on the old
    // stream must finish before calls on the new one reuse it; the pending
    // divergence records are reduced on the old stream first
    flush_ring(ctx);
    CHECK_LAUNCH(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->stream = static_cast<hipStream_t>(s);
    return FVK_OK;
}

fvk_status fvk_set_shift(fvk_ctx *ctx, double sigma) {
    if (!ctx) return FVK_EINVAL;
    if (!std::isfinite(sigma)) return fail(ctx, FVK_EINVAL, "shift must be finite");
    ctx->shift = sigma;
    return FVK_OK;
}

fvk_status fvk_get_shift(const fvk_ctx *ctx, double *sigma) {
    if (!ctx || !sigma) return FVK_EINVAL;
    *sigma = ctx->shift;
    return FVK_OK;
}

fvk_status fvk_set_params(fvk_ctx *ctx, double Gr, double Pr) {
    if (!ctx) return FVK_EINVAL;
    if (!(Gr > 0) || !(Pr > 0)) return fail(ctx, FVK_EINVAL, "Gr and Pr must be positive");
    ctx->Gr = Gr;
    ctx->Pr = Pr;
    set_coefs_from_params(ctx);
    return FVK_OK;
}

fvk_status fvk_set_coeffs(fvk_ctx *ctx, double nu, double kappa, double b) {
    if (!ctx) return FVK_EINVAL;
    ctx->co.nu = nu;
    ctx->co.kappa = kappa;
    ctx->co.b = b;
    return FVK_OK;
}

fvk_status fvk_set_terms(fvk_ctx *ctx, int mask) {
    if (!ctx) return FVK_EINVAL;
    if (mask & ~FVK_TERMS_ALL) return fail(ctx, FVK_EINVAL, "unknown term bits");
    Coefs &c = ctx->co;
    auto on = [&](int bit) { return (mask >> bit & 1) ? 1.0 : 0.0; };
    c.fb = on(0);
    c.fuv = on(1);
    c.fvu = on(2);
    for (int a = 0; a < 3; ++a) {
        c.fut[a] = on(3 + a);
        c.fvt[a] = on(6 + a);
    }
    c.terms = mask;
    return FVK_OK;
}

fvk_status fvk_set_precision(fvk_ctx *ctx, int prec) {
    if (!ctx) return FVK_EINVAL;
    if (prec != FVK_FP64 && prec != FVK_MIXED) return fail(ctx, FVK_EINVAL, "bad precision");
    ctx->prec = prec;
    return FVK_OK;
}

fvk_status fvk_set_tpf_path(fvk_ctx *ctx, int path) {
    if (!ctx) return FVK_EINVAL;
    if (path != FVK_TPF_AUTO && path != FVK_TPF_AXES && path != FVK_TPF_PLANES)
        return fail(ctx, FVK_EINVAL, "bad TPF path");
    if (path == FVK_TPF_PLANES && !tpf_plane_fits(ctx->n))
        return fail(ctx, FVK_EINVAL, "TPF plane kernels need 4 .. 128 cells per axis");
    ctx->tpf_path = path;
    return FVK_OK;
}

fvk_status fvk_get_tpf_path(const fvk_ctx *ctx, int *path) {
    if (!ctx || !path) return FVK_EINVAL;
    *path = tpf_uses_planes(ctx) ? FVK_TPF_PLANES : FVK_TPF_AXES;
    return FVK_OK;
}

fvk_status fvk_mixed_passes(const fvk_ctx *ctx, int *passes, int *calibrated) {
    if (!ctx) return FVK_EINVAL;
    if (passes) *passes = ctx->mixed_passes;
    if (calibrated) *calibrated = ctx->mixed_calibrated ? 1 : 0;
    return FVK_OK;
}

fvk_status fvk_set_simple(fvk_ctx *ctx, double tol, int max_passes) {
    if (!ctx) return FVK_EINVAL;
    if (!(tol > 0) || max_passes < 1 || max_passes > 100)
        return fail(ctx, FVK_EINVAL, "bad SIMPLE settings");
    flush_ring(ctx);   // the pending records are tested against the old tolerance
    ctx->simple_tol = tol;
    ctx->simple_cap = max_passes;
    ctx->mixed_calibrated = false;   // recalibrate the asynchronous mixed pass count
    ctx->mixed_passes = 2;
    return FVK_OK;
}

fvk_status fvk_layout(const fvk_ctx *ctx, size_t off[4], size_t *field_len, size_t *n_total) {
    if (!ctx) return FVK_EINVAL;
    const size_t F = size_t(ctx->geo.F);
    if (off)
        for (int f = 0; f < 4; ++f) off[f] = f * F;
    if (field_len) *field_len = F;
    if (n_total) *n_total = 4 * F;
    return FVK_OK;
}

fvk_status fvk_grid_axis(const fvk_ctx *ctx, int axis, double *faces, double *centres,
                         double *widths) {
    if (!ctx || axis < 0 || axis > 2) return FVK_EINVAL;
    const AxisHost &a = ctx->ax[axis];
    if (faces) std::memcpy(faces, a.f.data(), a.f.size() * 8);
    if (centres) std::memcpy(centres, a.c.data(), a.c.size() * 8);
    if (widths) std::memcpy(widths, a.h.data(), a.h.size() * 8);
    return FVK_OK;
}

const char *fvk_last_error(const fvk_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

fvk_status fvk_tridiag_eig(int n, const double *diag, const double *off, double *lam, double *Q) {
    if (n < 1 || !diag || !lam || !Q || (n > 1 && !off)) return FVK_EINVAL;
    return tridiag_eig(n, diag, off, lam, Q) == 0 ? FVK_OK : FVK_ENOCONV;
}

fvk_status fv_residual(fvk_ctx *ctx, const double *base, double *F, int project) {
    if (!ctx || !base || !F) return FVK_EINVAL;
    const Geo &g = ctx->geo;
    launch_residual(g, ctx->co, ctx->bc == FVK_SPAN_AA, base, F, ctx->stream);
    CHECK_LAUNCH(ctx);
    if (project) return fvk_project(ctx, F, F, 0);
    return FVK_OK;
}

fvk_status fv_jacvec(fvk_ctx *ctx, const double *base, const double *x, double *y,
                     int transpose) {
    if (!ctx || !base || !x || !y) return FVK_EINVAL;
    if (x == y) return fail(ctx, FVK_EINVAL, "x and y must not overlap");
    const Geo &g = ctx->geo;
    if (!transpose)
        launch_jacvec(g, ctx->co, ctx->bc == FVK_SPAN_AA, 0, base, x, y, y + 3 * g.F, ctx->stream);
    else
        launch_jacvec_T(g, ctx->co, ctx->bc == FVK_SPAN_AA, 0, base, x, x + 3 * g.F, y,
                        ctx->stream);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

fvk_status fvk_project(fvk_ctx *ctx, const double *x, double *y, int transpose) {
    if (!ctx || !x || !y) return FVK_EINVAL;
    const Geo &g = ctx->geo;
    Workspace &w = ctx->ws;
    hipStream_t st = ctx->stream;
    const long F = g.F;
    const int aa = ctx->bc == FVK_SPAN_AA;
    if (!transpose) {
        launch_ext_T(g, aa, x + 3 * F, w.vtmp + 3 * F, st);
        launch_zero_vel_walls(g, x, w.vtmp, st);
        CHECK_LAUNCH(ctx);
        int passes = 0;
        double dmax = 0.0;
        fvk_status s = simple_forward(ctx, w.vtmp, y, w.vtmp, nullptr, true, &passes, &dmax);
        launch_copy(y + 3 * F, w.vtmp + 3 * F, F, st);
        CHECK_LAUNCH(ctx);
        return s;
    }
    int passes = 0;
    double dmax = 0.0;
    fvk_status s = simple_transpose(ctx, x, w.vtmp, true, &passes, &dmax);
    if (s != FVK_OK) return s;
    launch_ext_T_T(g, aa, x + 3 * F, w.vtmp + 3 * F, st);
    launch_copy(y, w.vtmp, size_t(4) * F, st);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

fvk_status simple_krylov_vec(fvk_ctx *ctx, const double *base, const double *x, double *y,
                             double *p_out, int transpose, int *passes, double *max_div) {
    if (!ctx || !base || !x || !y) return FVK_EINVAL;
    if (x == y) return fail(ctx, FVK_EINVAL, "x and y must not overlap");
    const Geo &g = ctx->geo;
    Workspace &w = ctx->ws;
    hipStream_t st = ctx->stream;
    const long F = g.F;
    const int aa = ctx->bc == FVK_SPAN_AA;
    if (!transpose) {
        // momentum predictor + temperature RHS (eqs (11)-(12)), T part final;
        // with a shift the stencil returns (J + shift I) x
        Coefs cs = ctx->co;
        cs.sigma = ctx->shift;
        timing_begin(ctx, FVK_STAGE_JACVEC);
        launch_jacvec(g, cs, aa, 1, base, x, w.vtmp, y + 3 * F, st);
        timing_end(ctx, FVK_STAGE_JACVEC);
        CHECK_LAUNCH(ctx);
        const bool sync = passes || max_div;
        int k = 0;
        double dmax = 0.0;
        fvk_status s = simple_forward(ctx, w.vtmp, y, w.vtmp, p_out, sync, &k, &dmax);
        if (passes) *passes = k;
        if (max_div) *max_div = dmax;
        return s;
    }
    const bool sync = passes || max_div;
    int k = 0;
    double dmax = 0.0;
    fvk_status s = simple_transpose(ctx, x, w.vtmp, sync, &k, &dmax);
    if (passes) *passes = k;
    if (max_div) *max_div = dmax;
    if (s != FVK_OK) return s;
    Coefs cs = ctx->co;
    cs.sigma = ctx->shift;
    timing_begin(ctx, FVK_STAGE_JACVEC);
    launch_jacvec_T(g, cs, aa, 1, base, w.vtmp, x + 3 * F, y, st);
    timing_end(ctx, FVK_STAGE_JACVEC);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

fvk_status fvk_psi_projection(fvk_ctx *ctx, const double *vel, int axis, double *vproj,
                              double *psi) {
    if (!ctx || !vel || !vproj || axis < 0 || axis > 2) return FVK_EINVAL;
    const Geo &g = ctx->geo;
    Workspace &w = ctx->ws;
    hipStream_t st = ctx->stream;
    launch_div_plane(g, vel, w.div, axis, st);
    tpf_solve_plane(ctx, w.div, w.phi, axis, st);
    launch_correct_plane(g, vel, w.phi, vproj, axis, st);
    if (psi) launch_psi_lines(g, vproj, psi, axis, st);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

fvk_status fvk_simple_stats(fvk_ctx *ctx, double *max_div, int *n_unconverged) {
    if (!ctx) return FVK_EINVAL;
    flush_ring(ctx);
    CHECK_LAUNCH(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    double m = 0.0;
    int cnt = 0;
    HIPCHK(ctx, hipMemcpy(&m, ctx->ws.div_slots + 1, 8, hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(&cnt, ctx->ws.dev_counters, sizeof(int), hipMemcpyDeviceToHost));
    if (max_div) *max_div = m;
    if (n_unconverged) *n_unconverged = cnt;
    HIPCHK(ctx, hipMemset(ctx->ws.div_slots + 1, 0, 8));
    HIPCHK(ctx, hipMemset(ctx->ws.dev_counters, 0, sizeof(int)));
    return FVK_OK;
}

fvk_status fvk_multidot(fvk_ctx *ctx, const double *V, size_t ldv, int m, const double *w,
                        size_t n, double *out) {
    if (!ctx || !V || !w || !out || m < 1 || m > 1024 || n == 0) return FVK_EINVAL;
    const int nb = multidot_blocks(n);
    if (size_t(nb) * m > ctx->ws.red_len) return fail(ctx, FVK_EINVAL, "too many vectors");
    launch_multidot(V, ldv, m, w, n, ctx->ws.red, nb, ctx->stream);
    launch_reduce_partials(ctx->ws.red, nb, m, ctx->ws.dev_scalars + 8, 0, ctx->stream);
    CHECK_LAUNCH(ctx);
    return read_back(ctx, ctx->ws.dev_scalars + 8, out, m);
}

fvk_status fvk_multiaxpy(fvk_ctx *ctx, double *w, double alpha, const double *V, size_t ldv,
                         int m, const double *c, size_t n) {
    if (!ctx || !w || !V || !c || m < 1 || n == 0) return FVK_EINVAL;
    fvk_status s = write_coefs(ctx, c, m);
    if (s != FVK_OK) return s;
    launch_multiaxpy(w, alpha, 1.0, V, ldv, m, ctx->ws.coef_dev, n, ctx->stream);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

fvk_status fvk_axpby(fvk_ctx *ctx, double *y, double a, const double *x, double b, size_t n) {
    if (!ctx || !y || !x || n == 0) return FVK_EINVAL;
    launch_axpby(y, a, x, b, n, ctx->stream);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

fvk_status fvk_basis_rotate(fvk_ctx *ctx, double *V, size_t ldv, int m, const double *Q, int k,
                            size_t n) {
    if (!ctx || !V || !Q || m < 1 || k < 1 || k > m || m > 200 || n == 0) return FVK_EINVAL;
    fvk_status s = write_coefs(ctx, Q, size_t(m) * k);
    if (s != FVK_OK) return s;
    launch_basis_rotate(V, ldv, m, ctx->ws.coef_dev, k, n, ctx->stream);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

fvk_status arnoldi_step(fvk_ctx *ctx, const double *base, double *V, size_t ldv, int j,
                        double *h_col, int transpose) {
    if (!ctx || !base || !V || !h_col || j < 0 || j > 1000) return FVK_EINVAL;
    const size_t n = nvec(ctx);
    if (ldv < n) return fail(ctx, FVK_EINVAL, "ldv smaller than the vector length");
    const int m = j + 1;
    const int nb = multidot_blocks(n);
    if (size_t(nb) * m > ctx->ws.red_len || m + 2 > 1000)
        return fail(ctx, FVK_EINVAL, "Krylov dimension too large");
    double *wv = V + size_t(j + 1) * ldv;
    fvk_status s = simple_krylov_vec(ctx, base, V + size_t(j) * ldv, wv, nullptr, transpose,
                                     nullptr, nullptr);
    if (s != FVK_OK) return s;
    hipStream_t st = ctx->stream;
    double *h = ctx->ws.dev_scalars + 8;          // h[0..m)
    double *hr = ctx->ws.dev_scalars + 8 + 1001;  // re-orthogonalisation coefficients
    double *nrm = ctx->ws.dev_scalars + 4;
    // classical Gram-Schmidt, then one full re-orthogonalisation pass (CGS2)
    timing_begin(ctx, FVK_STAGE_ORTHO);
    launch_multidot(V, ldv, m, wv, n, ctx->ws.red, nb, st);
    launch_reduce_partials(ctx->ws.red, nb, m, h, 0, st);
    launch_multiaxpy(wv, 1.0, -1.0, V, ldv, m, h, n, st);
    launch_multidot(V, ldv, m, wv, n, ctx->ws.red, nb, st);
    launch_reduce_partials(ctx->ws.red, nb, m, hr, 0, st);
    launch_multiaxpy(wv, 1.0, -1.0, V, ldv, m, hr, n, st);
    launch_axpby(h, 1.0, hr, 1.0, m, st);
    launch_multidot(wv, ldv, 1, wv, n, ctx->ws.red, nb, st);
    launch_reduce_partials(ctx->ws.red, nb, 1, nrm, 0, st);
    launch_scale_inv_sqrt(wv, nrm, n, st);
    timing_end(ctx, FVK_STAGE_ORTHO);
    CHECK_LAUNCH(ctx);
    double nrm2 = 0.0;
    s = read_back(ctx, h, h_col, m);
    if (s != FVK_OK) return s;
    s = read_back(ctx, nrm, &nrm2, 1);
    if (s != FVK_OK) return s;
    h_col[j + 1] = std::sqrt(nrm2);
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
        return fail(ctx, FVK_EBREAKDOWN, "Arnoldi breakdown: |w| = 0 or not finite");
    return FVK_OK;
}

}  // extern "C"

// ---- lagged CGS2 ------------------------------------------------------------
// Slot j holds x (raw), orthogonal to v_0..v_{j-1} to first order; row j of
// H refers to x.  With d_q = v_q . x (q < j), alpha = x . x:
//   rho = |x|, s = d / rho, nu = sqrt(1 - |s|^2), v_j = (x / rho - V s) / nu,
// and x = rho (V s + nu v_j) moves rho s * (row j) into the rows above and
// scales row j by rho nu.  Returns the step's quantities for the caller.
namespace {

struct LagState {
    double rho, nu;
    std::vector<double> s;
};

// On a breakdown (x = 0, or x in the span of v_0..v_{j-1}) H is still
// corrected, with a zero row j: the Krylov space is invariant.
fvk_status lag_finalise(fvk_ctx *ctx, int j, double *H, int ldh, const double *d_xv,
                        double alpha, LagState &L) {
    const bool vanished = !(alpha > 0.0) || !std::isfinite(alpha);
    L.rho = vanished ? 0.0 : std::sqrt(alpha);
    L.s.assign(j, 0.0);
    double ss = 0.0;
    for (int q = 0; q < j && !vanished; ++q) {
        L.s[q] = d_xv[q] / L.rho;
        ss += L.s[q] * L.s[q];
    }
    const double nu2 = 1.0 - ss;
    const bool in_span = !vanished && !(nu2 > 1e-28);
    L.nu = (vanished || in_span) ? 0.0 : std::sqrt(nu2);
    for (int c = 0; c < j; ++c) {
        const double hjc = H[size_t(j) * ldh + c];
        if (hjc == 0.0) continue;
        for (int r = 0; r < j; ++r) H[size_t(r) * ldh + c] += L.rho * L.s[r] * hjc;
        H[size_t(j) * ldh + c] = hjc * L.rho * L.nu;
    }
    if (vanished) return fail(ctx, FVK_EBREAKDOWN, "Arnoldi breakdown: the new vector vanished");
    if (in_span) return fail(ctx, FVK_EBREAKDOWN, "Arnoldi breakdown: invariant subspace");
    return FVK_OK;
}

}  // namespace

extern "C" {

static fvk_status lagged_check(fvk_ctx *ctx, size_t ldv, int j) {
    const size_t n = nvec(ctx);
    if (ldv < n) return fail(ctx, FVK_EINVAL, "ldv smaller than the vector length");
    const int m2 = j + 2;   // rows v_0..v_{j-1}, slot j, slot j+1
    const int nb = multidot2_blocks(n);
    if (size_t(nb) * 2 * m2 > ctx->ws.red_len || 2 * m2 + 8 > 4096 || 2 * j > int(ctx->ws.coef_len))
        return fail(ctx, FVK_EINVAL, "Krylov dimension too large");
    return FVK_OK;
}

static fvk_status lagged_orthogonalise(fvk_ctx *ctx, double *V, size_t ldv, int j, double *H,
                                       int ldh);

fvk_status arnoldi_step_lagged(fvk_ctx *ctx, const double *base, double *V, size_t ldv, int j,
                               double *H, int ldh, int transpose) {
    if (!ctx || !base || !V || !H || j < 0 || ldh < j + 1) return FVK_EINVAL;
    fvk_status s = lagged_check(ctx, ldv, j);
    if (s != FVK_OK) return s;
    double *x = V + size_t(j) * ldv, *w = V + size_t(j + 1) * ldv;
    s = simple_krylov_vec(ctx, base, x, w, nullptr, transpose, nullptr, nullptr);
    if (s != FVK_OK) return s;
    return lagged_orthogonalise(ctx, V, ldv, j, H, ldh);
}

fvk_status arnoldi_step_lagged_applied(fvk_ctx *ctx, double *V, size_t ldv, int j, double *H,
                                       int ldh) {
    if (!ctx || !V || !H || j < 0 || ldh < j + 1) return FVK_EINVAL;
    fvk_status s = lagged_check(ctx, ldv, j);
    if (s != FVK_OK) return s;
    return lagged_orthogonalise(ctx, V, ldv, j, H, ldh);
}

fvk_status fvk_lincomb3(fvk_ctx *ctx, double *z, double a, const double *x, double b,
                        const double *y, double c, size_t n) {
    if (!ctx || !z || !x || !y || n == 0) return FVK_EINVAL;
    if (z == x || z == y) return fail(ctx, FVK_EINVAL, "z must not alias x or y");
    launch_lincomb3(z, a, x, b, y, c, n, ctx->stream);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

}  // extern "C"

// the lagged-CGS2 update of step j once slot j+1 holds the operator applied to
// slot j (see arnoldi_step_lagged)
static fvk_status lagged_orthogonalise(fvk_ctx *ctx, double *V, size_t ldv, int j, double *H,
                                       int ldh) {
    const size_t n = nvec(ctx);
    const int m2 = j + 2;
    const int nb = multidot2_blocks(n);
    double *x = V + size_t(j) * ldv, *w = V + size_t(j + 1) * ldv;
    fvk_status s = FVK_OK;
    hipStream_t st = ctx->stream;
    double *dots = ctx->ws.dev_scalars + 8;
    timing_begin(ctx, FVK_STAGE_ORTHO);
    launch_multidot2(V, ldv, m2, x, w, n, ctx->ws.red, nb, dots, st);
    timing_end(ctx, FVK_STAGE_ORTHO);
    CHECK_LAUNCH(ctx);
    std::vector<double> d(2 * m2);
    if ((s = read_back(ctx, dots, d.data(), d.size())) != FVK_OK) return s;
    // d[2q] = v_q . x, d[2q + 1] = v_q . (A x); q = j: x itself
    std::vector<double> dx(j), dt(j);
    for (int q = 0; q < j; ++q) {
        dx[q] = d[2 * q];
        dt[q] = d[2 * q + 1];
    }
    LagState L;
    if ((s = lag_finalise(ctx, j, H, ldh, dx.data(), d[2 * j], L)) != FVK_OK) return s;
    const double rho = L.rho, nu = L.nu;
    // A applied to the unit vector x/rho: t = V^T (A x) / rho, beta = (x . A x) / rho^2
    std::vector<double> t(j);
    double st_ = 0.0;
    for (int q = 0; q < j; ++q) {
        t[q] = dt[q] / rho;
        st_ += L.s[q] * t[q];
    }
    const double beta = d[2 * j + 1] / (rho * rho);
    // A V_j s = V_{j+1} g with the corrected columns 0..j-1
    std::vector<double> g(j + 1, 0.0), h(j + 1), u(j + 1);
    for (int r = 0; r <= j; ++r)
        for (int c = 0; c < j; ++c) g[r] += H[size_t(r) * ldh + c] * L.s[c];
    for (int r = 0; r < j; ++r) h[r] = (t[r] - g[r]) / nu;
    h[j] = ((beta - st_) / nu - g[j]) / nu;
    for (int r = 0; r <= j; ++r) {
        H[size_t(r) * ldh + j] = h[r];
        u[r] = g[r] / nu + h[r];
    }
    H[size_t(j + 1) * ldh + j] = 1.0;
    // v_j = x / (rho nu) - V s / nu;
    // w' = A x / (rho nu) - u_j x / (rho nu) - V (u - s u_j / nu)
    std::vector<double> coef(2 * j);
    for (int q = 0; q < j; ++q) {
        coef[q] = -L.s[q] / nu;
        coef[j + q] = -(u[q] - L.s[q] * u[j] / nu);
    }
    if (j > 0 && (s = write_coefs(ctx, coef.data(), coef.size())) != FVK_OK) return s;
    const double c1 = 1.0 / (rho * nu);
    timing_begin(ctx, FVK_STAGE_ORTHO);
    launch_update2(x, w, V, ldv, j, ctx->ws.coef_dev, ctx->ws.coef_dev + j, c1, c1, -u[j] * c1, n,
                   st);
    timing_end(ctx, FVK_STAGE_ORTHO);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

extern "C" {

fvk_status arnoldi_finish(fvk_ctx *ctx, double *V, size_t ldv, int j, double *H, int ldh) {
    if (!ctx || !V || !H || j < 0 || (j > 0 && ldh < j)) return FVK_EINVAL;
    const size_t n = nvec(ctx);
    if (ldv < n) return fail(ctx, FVK_EINVAL, "ldv smaller than the vector length");
    const int m = j + 1;
    const int nb = multidot_blocks(n);
    if (size_t(nb) * m > ctx->ws.red_len || m + 8 > 4096 || j > int(ctx->ws.coef_len))
        return fail(ctx, FVK_EINVAL, "Krylov dimension too large");
    double *x = V + size_t(j) * ldv;
    hipStream_t st = ctx->stream;
    double *dots = ctx->ws.dev_scalars + 8;
    launch_multidot(V, ldv, m, x, n, ctx->ws.red, nb, st);
    launch_reduce_partials(ctx->ws.red, nb, m, dots, 0, st);
    CHECK_LAUNCH(ctx);
    std::vector<double> d(m);
    fvk_status s = read_back(ctx, dots, d.data(), m);
    if (s != FVK_OK) return s;
    LagState L;
    if ((s = lag_finalise(ctx, j, H, ldh, d.data(), d[j], L)) != FVK_OK) return s;
    std::vector<double> coef(j);
    for (int q = 0; q < j; ++q) coef[q] = -L.s[q] / L.nu;
    if (j > 0 && (s = write_coefs(ctx, coef.data(), coef.size())) != FVK_OK) return s;
    launch_multiaxpy(x, 1.0 / (L.rho * L.nu), 1.0, V, ldv, j, ctx->ws.coef_dev, n, st);
    CHECK_LAUNCH(ctx);
    return FVK_OK;
}

}  // extern "C"
