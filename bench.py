#!/usr/bin/env python
"""Throughput of the Krylov-vector hot path on one MI355X.

Workload (one step): the 100^3 throughput configuration -- tanh-stretched grid
(beta = 1.5), Pr = 0.71, Gr = 1e6, a seeded divergence-free synthetic base
flow, and 64 seeded unit-norm Krylov vectors in the constraint subspace; one
step applies simple_krylov_vec (Jacobian stencil, SIMPLE pass with the TPF
Poisson solve, temperature projection) to all 64 vectors for both spanwise
wall variants (conducting CC and insulated AA), i.e. 128 Krylov vectors, all
FP64.  Inputs are resident in device memory before the timed region.  The two
wall variants are independent problems, each with its own library context;
on grids of up to 160^3 cells, where one problem's kernels do not fill the
GPU, each context runs on its own HIP stream so that their kernels overlap
(--streams 1 serialises them).  The timed region is bracketed by device
synchronisations and timed on the host clock.

Prints one JSON line: value = Krylov vectors per second, a roofline entry for
the dominant kernel (timed live with HIP events on the library's stream, one
context at a time so that the kernel durations are those of the kernels
alone) and a CPU baseline of the oracle on a bounded sample of the same
workload.  Besides the headline 100^3 value the line carries the other half
of the metric: `n256` (FP64, mixed-precision and adjoint rates at 256^3 with
their per-stage roofline) and `lambda_error` (the rightmost eigenvalues at
100^3 in FP64 and in mixed precision, and their difference).

Usage: python bench.py [--steps K] [--warmup W] [--n N] [--nvec M]
       [--streams S] [--tpf auto|axes|planes] [--no-cpu-baseline] [--no-extra]
       [--no-eig] [--no-256]
       (--tpf planes: the opt-in plane kernels of the TPF solve, for comparison)
       python bench.py --copy-calibration          (a 2 GiB device copy, for
                                                    rocprofv3 --pmc scaling)
       python bench.py --ingest-pmc FETCH WRITE CFETCH CWRITE
           reads four rocprofv3 --pmc output folders (FETCH_SIZE and
           WRITE_SIZE of a bench run, then of the copy calibration) and
           writes profiles/traffic.json: HBM bytes per launch of each
           kernel of the Krylov vector (stencil, divergence-forming and
           plain transforms, correction), scaled so the copy reads and
           writes exactly its size, each tagged with a hash of its source
           file (a later edit of the source makes the entry stale and
           bench.py reports null for it).
"""
import csv
import glob
import hashlib
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Krylov vectors/s at 100^3 & 256^3 (FP64 vs mixed+adjoint) at stated "
          "λ error")
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
COPY_BYTES = 1 << 31         # copy calibration: 2 GiB read + 2 GiB written
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_1905_11601_amd", "csrc")


def transform_kernel(n):
    """Name of the per-axis transform kernel the library runs for n cells (the
    register-resident variant for 193..256 cells, else the streaming one)."""
    ne = n - n // 2
    return "k_axis_res" if 96 < ne <= 128 else "k_axis_sym"


def transform_work(n):
    """(flops, bytes) of one even/odd axis transform of an n^3 FP64 array:
    two half-size products per pencil, each input and output value moved once."""
    ne, no = n - n // 2, n // 2
    return 2.0 * (ne * ne + no * no) * n * n, 16.0 * n ** 3


def stage_kernels(n, planes=False):
    """stage -> (kernels, source file, algorithmic bytes per launch, flops per
    launch) of one FP64 Krylov vector at n^3 (planes: the opt-in plane
    kernels of the TPF solve, else the per-axis ones)."""
    npts, ncell = (n + 2) ** 3, n ** 3
    f1, _ = transform_work(n)
    out = {"jacvec": (("k_jac_tiled",), "kernels_stencil.hip", stencil_bytes_per_point() * npts,
                      0.0),
           # reads v* (3 fields) and phi on the cells, writes v (3 fields)
           # on every stored point (walls zeroed); no divergence store on the
           # last pass of a call
           "correct": (("k_correct<",), "kernels_stencil.hip", (3 + 1) * 8 * ncell + 3 * 8 * npts,
                       0.0)}
    if planes:
        # divergence from the faces (3 reads) + x and y forward transforms,
        # one write; then z forward / scale / z inverse and y / x inverse,
        # each one read and one write and two transforms
        out["div"] = (("k_plane_fwd",), "kernels_tpf_plane.hip", 32.0 * ncell, 2 * f1)
        out["transform"] = (("k_plane_mid", "k_plane_inv"), "kernels_tpf_plane.hip",
                            16.0 * ncell, 2 * f1)
    else:
        out["div"] = (("k_axis_sym:div",), "kernels_tpf.hip", 32.0 * ncell, f1)
        out["transform"] = ((transform_kernel(n),), "kernels_tpf.hip", 16.0 * ncell, f1)
    return out


def roof_of(work_bytes, flops, seconds):
    """Roofline entry of one launch: bound by whichever of HBM and FP64 MFMA
    is tighter for its bytes and flops."""
    if flops and flops / (FP64_PEAK_TFS * 1e12) > work_bytes / (HBM_PEAK_GBS * 1e9):
        a = flops / seconds / 1e12
        return {"bound": "mfma", "achieved": a, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                "frac": a / FP64_PEAK_TFS}
    a = work_bytes / seconds / 1e9
    return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": a / HBM_PEAK_GBS}


FP64_PEAK_TFS = 78.6         # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFS = 157.3        # MI355X dense FP32 matrix


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(fvk, torch, n, nvec, bc, prec, stream):
    """Context on `stream`, base flow and nvec projected unit inputs, all made
    on that stream (and finished before returning)."""
    from paper_1905_11601_amd import inputs
    with torch.cuda.stream(stream):
        ctx = fvk.Ctx(n, grid=fvk.TANH, s=1.5, span_bc=bc, Gr=1e6, Pr=0.71, prec=prec,
                      stream=stream)
        f, c, h = ctx.coords()
        base = torch.as_tensor(inputs.synthetic_base(f, c, h, bc)).cuda()
        X = torch.empty((nvec,) + ctx.shape4, dtype=torch.float64, device="cuda")
        for q in range(nvec):
            raw = torch.as_tensor(inputs.random_fields(ctx.n, 2000 + q)).cuda()
            ctx.project(raw, out=X[q])
            ctx.normalize(X[q])
    stream.synchronize()
    return ctx, base, X


def stencil_bytes_per_point():
    # jacvec: reads base (4 fields) + x (4 fields), writes the momentum
    # predictor (3 fields) + projected T (1 field), every stored point, FP64
    return (8 + 4) * 8


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def copy_calibration():
    import torch
    n = COPY_BYTES // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 3}))


def _forms_divergence(kernel_name):
    """True for the x-axis transform instances that read the velocity fields
    and form the divergence (last template argument 1 or 2): they belong to
    the divergence stage, not to the plain transforms."""
    if "k_axis_sym<" not in kernel_name:
        return False
    head = kernel_name[kernel_name.index("k_axis_sym<") + len("k_axis_sym<"):]
    args = head[:head.index(">")].split(",")
    return len(args) == 9 and args[-1].strip() != "0"


def _matches(kernel_name, part):
    """Kernel selector of stage_kernels: a name part; "k_axis_sym:div" is the
    divergence-forming instance of k_axis_sym, a plain k_axis_sym part
    excludes those instances."""
    if part == "k_axis_sym:div":
        return _forms_divergence(kernel_name)
    return part in kernel_name and not _forms_divergence(kernel_name)


def _pmc_rows(folder, counter, part):
    """Per-dispatch values (bytes) of `counter` for the kernels selected by
    `part` (see _matches), from a rocprofv3 --pmc csv folder (values in KiB)."""
    out = []
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] == counter and _matches(row["Kernel_Name"], part):
                    out.append(float(row["Counter_Value"]) * 1024.0)
    return out


def ingest_pmc(fetch_dir, write_dir, cfetch_dir, cwrite_dir, n):
    # the copy is the largest dispatch of the calibration run
    cf = max(_pmc_rows(cfetch_dir, "FETCH_SIZE", ""))
    cw = max(_pmc_rows(cwrite_dir, "WRITE_SIZE", ""))
    kf, kw = COPY_BYTES / cf, COPY_BYTES / cw
    rec = {"grid": n, "copy_fetch_bytes_raw": cf, "copy_write_bytes_raw": cw,
           "fetch_scale": kf, "write_scale": kw, "kernels": {}}
    for stage, (parts, src, nbytes, _) in stage_kernels(n).items():
        for part in parts:
            fetch = _pmc_rows(fetch_dir, "FETCH_SIZE", part)
            write = _pmc_rows(write_dir, "WRITE_SIZE", part)
            if not fetch or not write:
                raise SystemExit(f"no {part} dispatches in the pmc folders")
            f_avg, w_avg = sum(fetch) / len(fetch), sum(write) / len(write)
            rec["kernels"][part] = {
                "stage": stage, "source": os.path.join("paper_1905_11601_amd", "csrc", src),
                "source_sha256": source_hash(os.path.join(CSRC, src)),
                "dispatches": [len(fetch), len(write)],
                "fetch_bytes_raw": f_avg, "write_bytes_raw": w_avg,
                "read_bytes_per_launch": f_avg * kf, "write_bytes_per_launch": w_avg * kw,
                "traffic_bytes_per_launch": f_avg * kf + w_avg * kw,
                "algorithmic_bytes_per_launch": nbytes}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def traffic_entry(n, stage, planes=False):
    """Measured HBM bytes per launch of the kernels of `stage` (their mean),
    or None when no measurement matches this grid and the current sources."""
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    parts, src, _, _ = stage_kernels(n, planes)[stage]
    if rec.get("grid") != n:
        return None
    vals = []
    for part in parts:
        k = rec.get("kernels", {}).get(part)
        if not k or k.get("source_sha256") != source_hash(os.path.join(CSRC, src)):
            return None
        vals.append(k["traffic_bytes_per_launch"])
    return sum(vals) / len(vals)


def host_info():
    """Host CPU facts for the baseline: logical CPUs visible to this process
    and the CPU model (lscpu)."""
    import subprocess
    info = {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core"):
                info[key.strip()] = val.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(n, min_seconds, one_thread_seconds):
    """The oracle on the host cores: simple_krylov_vec of the same workload on
    a bounded sample (as many calls as fit in min_seconds, CC walls), then the
    same with one thread."""
    import torch
    from oracle import ops
    from oracle.grid import Grid, TANH
    from oracle.krylov import Oracle
    from paper_1905_11601_amd import inputs
    g = Grid(n, kind=TANH, s=1.5)
    orc = Oracle(g, ops.Params(1e6, 0.71), 0)
    f = tuple(a.f for a in g.ax)
    c = tuple(a.c for a in g.ax)
    h = tuple(a.h for a in g.ax)
    U = torch.as_tensor(inputs.synthetic_base(f, c, h, 0))
    xs = []
    ndistinct = 16   # inputs reused cyclically (host memory)
    for q in range(ndistinct):
        x = orc.project(torch.as_tensor(inputs.random_fields(g.n, 2000 + q)))
        xs.append(x / torch.linalg.norm(x))
    def rate(seconds):
        orc.krylov_vec(U, xs[0])                  # warm-up
        t0 = time.perf_counter()
        calls = 0
        while True:
            orc.krylov_vec(U, xs[calls % ndistinct])
            calls += 1
            dt = time.perf_counter() - t0
            if dt >= seconds and calls >= 4:
                return calls, dt

    threads = torch.get_num_threads()
    calls, dt = rate(min_seconds)
    out = {"value": calls / dt, "unit": "Krylov vectors/s", "cores": threads, "kind": "oracle",
           "sample": f"{calls} simple_krylov_vec calls at {n}^3 ({ndistinct} distinct seeded "
                     f"unit inputs, cyclic), CC walls, PyTorch CPU FP64 oracle on {threads} "
                     f"threads, {dt:.1f} s",
           "host": host_info()}
    if one_thread_seconds > 0:
        torch.set_num_threads(1)
        try:
            c1, d1 = rate(one_thread_seconds)
        finally:
            torch.set_num_threads(threads)
        out["one_thread"] = {"value": c1 / d1, "unit": "Krylov vectors/s", "cores": 1,
                             "sample": f"{c1} calls, {d1:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--nvec", type=int, default=64)
    ap.add_argument("--streams", type=int, default=0, choices=(0, 1, 2),
                    help="1: both wall variants on one stream; 2: one stream each; "
                         "0 (default): 2 up to 160^3 cells, else 1")
    ap.add_argument("--tpf", choices=("auto", "axes", "planes"), default="auto",
                    help="kernels of the TPF solve (fvk_set_tpf_path)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="oracle baseline: time budget of the all-threads sample")
    ap.add_argument("--cpu-one-thread-seconds", type=float, default=8.0)
    ap.add_argument("--no-256", action="store_true",
                    help="skip the 256^3 leg (FP64, mixed and adjoint rates at 256^3)")
    ap.add_argument("--nvec-256", type=int, default=8)
    ap.add_argument("--no-eig", action="store_true",
                    help="skip the eigenvalue-error leg (FP64 vs mixed Krylov-Schur)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the mixed-precision, adjoint and Arnoldi-step rates")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--ingest-pmc", nargs=4, metavar="DIR")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc, n=args.n)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not an implementation", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1905_11601_amd as fvk

    n, nvec = args.n, args.nvec
    nstreams = args.streams or (2 if n <= 160 else 1)
    log(f"setup {n}^3, {nvec} vectors x 2 wall variants on {nstreams} stream(s)")
    if nstreams == 2:
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]   # default priority
    else:
        streams = [torch.cuda.current_stream()] * 2
    runs = [make_inputs(fvk, torch, n, nvec, bc, fvk.FP64, st)
            for bc, st in zip((fvk.CC, fvk.AA), streams)]
    if args.tpf != "auto":
        for ctx, _, _ in runs:
            ctx.set_tpf_path(fvk.TPF_AXES if args.tpf == "axes" else fvk.TPF_PLANES)
    Ys = []
    for (_, _, X), st in zip(runs, streams):
        with torch.cuda.stream(st):
            Ys.append(torch.empty_like(X))

    def submit(q, r):
        ctx, base, X = runs[r]
        ctx.simple_krylov_vec(base, X[q], out=Ys[r][q])

    def step():
        # the two problems' vectors interleaved, so that both streams have
        # work queued at any time
        for q in range(nvec):
            for r in range(2):
                submit(q, r)

    for ctx, _, _ in runs:
        ctx.simple_stats()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = wall * 1e3
    nvec_total = 2 * nvec * args.steps
    value = nvec_total / wall
    max_div = 0.0
    for ctx, _, _ in runs:
        d, bad = ctx.simple_stats()
        if bad:
            raise SystemExit(f"{bad} Krylov vectors failed the divergence test")
        max_div = max(max_div, d)

    # ---- roofline of the dominant kernel: the same vectors again with
    # HIP-event stage timing on each context's stream, one context at a time
    # (no kernels of the other problem running alongside)
    stages = {}
    for r, (ctx, _, _) in enumerate(runs):
        ctx.set_timing(("jacvec", "div", "transform", "correct"))
        for _ in range(args.steps):
            for q in range(nvec):
                submit(q, r)
        for k, (ms, cnt) in ctx.timing_read().items():   # synchronises
            a = stages.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += cnt
        ctx.set_timing(())
    log("stage times (ms total / launches): " + json.dumps(stages))
    ctx0 = runs[0][0]
    npts = (n + 2) ** 3
    ncell = n ** 3
    per = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    dominant = max(("jacvec", "transform", "correct", "div"), key=lambda k: stages[k][0])
    kernels = stage_kernels(n, planes=args.tpf == "planes")
    parts, src, nbytes, flops = kernels[dominant]
    roof = {"kernel": " + ".join(p.split(":")[0] for p in parts) + f" ({dominant} stage)"}
    roof.update(roof_of(nbytes, flops, per[dominant] * 1e-3))
    roof.update({"traffic": traffic_entry(n, dominant, args.tpf == "planes"),
                 "traffic_unit": "bytes per launch",
                 "algorithmic_bytes_per_launch": nbytes, "flops_per_launch": flops,
                 "per_launch_us": per[dominant] * 1e3, "source": src})
    roof["stages"] = {k: dict(roof_of(kernels[k][2], kernels[k][3], per[k] * 1e-3),
                              us=per[k] * 1e3, kernels=list(kernels[k][0]))
                      for k in kernels if stages.get(k, (0, 0))[1]}
    roof["stages_us_per_launch"] = {k: v * 1e3 for k, v in per.items() if stages[k][1]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Krylov vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"simple_krylov_vec, {n}^3 tanh-stretched (beta 1.5) staggered FV "
                               f"cube, Pr 0.71, Gr 1e6, synthetic divergence-free base flow, "
                               f"{nvec} seeded unit Krylov vectors x (CC, AA) spanwise walls, FP64",
                   "grid": n, "vectors_per_step": 2 * nvec,
                   "parallelism": f"single GPU, {nstreams} stream(s)",
                   "max_div_after_simple": max_div},
        "roofline": roof,
        "wall_s": wall,
    }
    if not args.no_extra:
        log("extra rates")
        out["extra"] = extra_rates(fvk, torch, runs, args)
    if not args.no_eig:
        log("eigenvalue error: FP64 vs mixed Krylov-Schur")
        out["lambda_error"] = eigen_leg(fvk, torch, runs[0][0], runs[0][1])
    del runs, Ys
    torch.cuda.empty_cache()
    if not args.no_256 and n != 256:
        log("256^3 leg")
        out["n256"] = leg_256(fvk, torch, args.nvec_256, max(1, min(args.steps, 3)))
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds, args.cpu_one_thread_seconds)
    print(json.dumps(out))


def stage_roofline(per_us, n):
    """Roofline fractions of the stages of one FP64 Krylov vector at n^3 from
    their average launch durations (us): the Jacobian stencil and the
    correction against HBM (algorithmic bytes), the axis transforms against
    whichever of HBM and FP64 MFMA is tighter for their size."""
    npts, ncell = (n + 2) ** 3, n ** 3
    out = {}
    for k, nbytes in (("jacvec", stencil_bytes_per_point() * npts),
                      ("correct", (3 + 1) * 8 * ncell + 3 * 8 * npts)):
        if per_us.get(k):
            gbs = nbytes / (per_us[k] * 1e-6) / 1e9
            out[k] = {"us": per_us[k], "GB/s": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}
    if per_us.get("transform"):
        flops, nbytes = transform_work(n)
        t = per_us["transform"] * 1e-6
        out["transform"] = {"us": per_us["transform"], "GB/s": nbytes / t / 1e9,
                            "frac_hbm": nbytes / t / 1e9 / HBM_PEAK_GBS,
                            "TFLOP/s": flops / t / 1e12,
                            "frac_fp64_mfma": flops / t / 1e12 / FP64_PEAK_TFS}
    return out


def leg_256(fvk, torch, nvec, reps):
    """The 256^3 half of the metric: FP64, mixed-precision and transposed
    (adjoint) Krylov-vector rates on nvec seeded unit inputs for each wall
    variant (one context and one stream each, vectors back to back, as an
    Arnoldi or GMRES iteration issues them), and the per-stage roofline of the
    FP64 vector from HIP events."""
    from paper_1905_11601_amd import inputs
    n = 256
    raws = [torch.as_tensor(inputs.random_fields((n, n, n), 2000 + q)) for q in range(nvec)]
    kinds = (("fp64", fvk.FP64, False), ("mixed", fvk.MIXED, False),
             ("fp64_adjoint", fvk.FP64, True), ("mixed_adjoint", fvk.MIXED, True))
    acc = {k: [0, 0.0] for k, _, _ in kinds}
    stages = {}
    max_div = 0.0
    n_bad = 0
    records = {}
    for bc in (fvk.CC, fvk.AA):
        ctx = fvk.Ctx(n, grid=fvk.TANH, s=1.5, span_bc=bc, Gr=1e6, Pr=0.71)
        f, c, h = ctx.coords()
        base = torch.as_tensor(inputs.synthetic_base(f, c, h, bc)).cuda()
        X = torch.empty((nvec,) + ctx.shape4, dtype=torch.float64, device="cuda")
        for q in range(nvec):
            ctx.project(raws[q].cuda(), out=X[q])
            ctx.normalize(X[q])
        Y = torch.empty_like(X)
        ctx.simple_stats()

        def run(tr):
            for q in range(nvec):
                ctx.simple_krylov_vec(base, X[q], out=Y[q], transpose=tr)

        wall = "CC" if bc == fvk.CC else "AA"
        for key, prec, tr in kinds:
            ctx.set_precision(prec)
            run(tr)
            ms = timed(torch, lambda: run(tr), reps)
            acc[key][0] += nvec
            acc[key][1] += ms / 1e3
            if not tr:
                # the divergence records of this precision's asynchronous calls
                d, bad = ctx.simple_stats()
                records[f"{wall}_{key}"] = {"max_div": d, "calls_above_tol": bad,
                                            "passes": (ctx.mixed_passes()[0]
                                                       if prec == fvk.MIXED else 1)}
                max_div = max(max_div, d)
                n_bad += bad
        ctx.set_precision(fvk.FP64)
        ctx.set_timing(("jacvec", "div", "transform", "correct"))
        for _ in range(reps):
            run(False)
        for k, (ms, cnt) in ctx.timing_read().items():
            a = stages.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += cnt
        ctx.set_timing(())
        ctx.simple_stats()
        del X, Y, base
        ctx.close()
        torch.cuda.empty_cache()
    per_us = {k: 1e3 * v[0] / v[1] for k, v in stages.items() if v[1]}
    rates = {f"{k}_vec_per_s": v[0] / v[1] for k, v in acc.items()}
    return {"grid": n, "vectors_per_wall_variant": nvec, "walls": ["CC", "AA"],
            "streams": 1, **rates, "max_div_after_simple": max_div,
            "calls_above_simple_tol": n_bad, "divergence_records": records,
            "stages_us_per_launch": per_us, "roofline": stage_roofline(per_us, n)}


def eigen_leg(fvk, torch, ctx, base, k=4, m=100, tol=1e-9):
    """The eigenvalue accuracy the rates are quoted at: the k rightmost
    eigenvalues of the 100^3 CC problem by Krylov-Schur (Krylov dimension m)
    in FP64 and in mixed precision from the same start vector, their Ritz
    residuals, and the largest mixed-vs-FP64 difference."""
    import numpy as np
    from paper_1905_11601_amd import inputs
    from paper_1905_11601_amd.eigs import krylov_schur
    with torch.cuda.stream(ctx.stream):
        v0 = ctx.project(torch.as_tensor(inputs.random_fields(ctx.n, 5000)).cuda())
        out = {"workload": f"{k} rightmost eigenvalues, {ctx.n[0]}^3 CC, Krylov dimension {m}, "
                           f"Ritz residual tolerance {tol:g}, start vector seed 5000"}
        lams = {}
        for name, prec in (("fp64", fvk.FP64), ("mixed", fvk.MIXED)):
            ctx.set_precision(prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = krylov_schur(ctx, base, k=k, m=m, v0=v0, tol=tol, max_restarts=400,
                             vectors=False)
            torch.cuda.synchronize()
            lams[name] = r.lam
            out[name] = {"eigenvalues": [[float(v.real), float(v.imag)] for v in r.lam],
                         "ritz_residual_max": float(np.max(r.res)), "converged": r.converged,
                         "krylov_vectors": r.nvec, "seconds": time.perf_counter() - t0}
        ctx.set_precision(fvk.FP64)
    d = [float(np.min(np.abs(lams["fp64"] - l))) for l in lams["mixed"]]
    out["mixed_vs_fp64_max_abs"] = max(d)
    out["mixed_vs_fp64_max_rel"] = max(d) / float(np.abs(lams["fp64"]).max())
    return out


def timed(torch, fn, reps):
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def extra_rates(fvk, torch, runs, args):
    """Mixed-precision and transposed (adjoint) Krylov-vector rates on the same
    vectors, and the Arnoldi-step rate at Krylov dimension 40: one context,
    one stream, vectors one after the other."""
    with torch.cuda.stream(runs[0][0].stream):
        return _extra_rates(fvk, torch, runs, args)


def _extra_rates(fvk, torch, runs, args):
    ctx, base, X = runs[0]
    nvec = X.shape[0]
    Y = torch.empty_like(X)
    res = {}

    def run(transpose):
        for q in range(nvec):
            ctx.simple_krylov_vec(base, X[q], out=Y[q], transpose=transpose)

    run(False)
    res["fp64_vec_per_s"] = nvec / (timed(torch, lambda: run(False), 2) / 1e3)
    ref = Y.clone()
    ctx.set_precision(fvk.MIXED)
    run(False)
    res["mixed_vec_per_s"] = nvec / (timed(torch, lambda: run(False), 2) / 1e3)
    res["mixed_max_rel_diff_vs_fp64"] = float(((Y - ref).abs().max() / ref.abs().max()).item())
    run(True)
    res["mixed_adjoint_vec_per_s"] = nvec / (timed(torch, lambda: run(True), 2) / 1e3)
    ctx.set_precision(fvk.FP64)
    run(True)
    res["fp64_adjoint_vec_per_s"] = nvec / (timed(torch, lambda: run(True), 2) / 1e3)
    m = 40
    V = torch.zeros((m + 1, ctx.N), dtype=torch.float64, device="cuda")
    V[0] = X[0].reshape(-1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(m):
        ctx.arnoldi_step(base, V, j)
    torch.cuda.synchronize()
    res["arnoldi_steps_per_s_m40"] = m / (time.perf_counter() - t0)
    # the same m steps with the lagged re-orthogonalisation (two passes over
    # the basis per step), completed by arnoldi_finish
    import numpy as np
    V.zero_()
    V[0] = X[0].reshape(-1)
    H = np.zeros((m + 1, m))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(m):
        ctx.arnoldi_step_lagged(base, V, j, H)
    ctx.arnoldi_finish(V, m, H)
    torch.cuda.synchronize()
    res["arnoldi_lagged_steps_per_s_m40"] = m / (time.perf_counter() - t0)
    return res


if __name__ == "__main__":
    main()
