"""Throughput of the batched, autograd FWI gradient on one MI355X.

One step = the whole hot path over one batch of synthetic input, inputs
resident in HBM: model prep, forward sweep of every shot with sqrt(nt)
snapshots and boundary strips, time-integral misfit and adjoint source
(eq. (2)), the fused backward sweep (source-wavefield reconstruction, adjoint
propagation, zero-lag imaging, eq. (1) illumination), the per-shot Hessian
epilogue and the preconditioned gradient, driven through torch.autograd
(J.backward()).

Workloads (--workload):
  offset   (default) 2048x768 layered model at dx = 6.25 m, 32 shots, 1024
           receivers each, nt = 8000, dt = 0.5 ms, Ricker 15 Hz; H1 and the
           offset diagonal |h| <= 16; sub-offset Hessian preconditioner (the
           largest configuration, the batched autograd preconditioned
           gradient of section 3)
  layered  1024x384 at dx = 12.5 m, 64 shots, 512 receivers each, nt = 4000,
           dt = 1 ms, Ricker 8 Hz; H1 and the offset diagonal |h| <= 16;
           shot-scaling preconditioner
  ragged   the 1024x384 model, 256 shots of 128..1024 receivers and nt
           2000..6000; H1; shot-scaling preconditioner

Prints one JSON line.  `value` is shot-gradients per second; the line also
carries Gcell-updates/s, the roofline of the dominant kernel (the fused
reverse step), the plain per-shot GPU path on a subset of shots, and the FP64
oracle timed on the host's cores on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["layered", "ragged", "offset"], default="offset")
    ap.add_argument("--shots", type=int, default=0, help="use only the first SHOTS shots (0 = all)")
    ap.add_argument("--plain-shots", type=int, default=4)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="time steps of each worker's oracle sample (0 = about 15 s of work per worker)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle worker processes (0 = the cores this process may use, at most 16)")
    ap.add_argument("--nt", type=int, default=0,
                    help="shorten every record to NT samples (counter-collection runs; 0 = full)")
    ap.add_argument("--ext", type=int, default=-1,
                    help="also time the offset-extended image for |h| <= EXT against the plain gradient call")
    ap.add_argument("--gn", action="store_true",
                    help="also time the Gauss-Newton Hessian-vector product against the plain gradient call")
    ap.add_argument("--exact-diag", type=int, default=0,
                    help="also time the offset diagonal with the exact receiver term on the first "
                         "--exact-shots shots and EXACT_DIAG of their receivers (band to 4 f_peak)")
    ap.add_argument("--exact-shots", type=int, default=2)
    ap.add_argument("--exact-sif", type=int, default=0,
                    help="runs in flight of the exact offset diagonal (0 = the library's default)")
    ap.add_argument("--exact-dft", choices=["both", "fp32", "bf16x3"], default="both",
                    help="DFT arithmetic(s) timed for the exact offset diagonal")
    ap.add_argument("--exec", type=str, default="",
                    help="pin the launch configuration instead of autotuning: "
                         "S,TZ,graph_steps,prefetch,prefetch_reverse[,S_rev,TZ_rev,reverse_steps,forward_steps"
                         "[,graph_branches]]")
    return ap.parse_args()


def reverse_bytes_per_shot_step(grid, nrec):
    """Algorithmic HBM bytes of one fused reverse step of one shot (FP32):
    model cells read u[m], u[m-1], lam[m+1], lam[m+2], w, g, E and write
    u[m-2], lam[m], g, E (44 B); the 4-cell strip ring reads its strip value
    and writes u besides the adjoint update (24 B); other sponge cells only
    advance the adjoint wavefield (16 B); receivers read psi (4 B)."""
    nz, nx, N = grid.nz, grid.nx, grid.nsponge
    model = nz * nx
    padded = (nz + 2 * N) * (nx + 2 * N)
    ring = 8 * (nz + nx)
    return 44 * model + 24 * ring + 16 * (padded - model - ring) + 4 * nrec


def forward_bytes_per_shot_step(grid, nrec, K):
    """Forward step in increment form: read u[n], d[n], w; write u[n+1],
    d[n+1] (20 B per padded cell); strip ring 4 B; snapshot pair every K
    steps 8 B per model cell; receivers 4 B."""
    nz, nx, N = grid.nz, grid.nx, grid.nsponge
    model = nz * nx
    padded = (nz + 2 * N) * (nx + 2 * N)
    ring = 8 * (nz + nx)
    return 20 * padded + 4 * ring + 8 * model / K + 4 * nrec


def kernel_hash():
    h = hashlib.sha256()
    for f in ("fwi_kernels.hip", "fwi_internal.h"):
        with open(os.path.join(ROOT, "paper_1406_1864_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# synthetic.WORKLOADS name of each benchmark workload
WNAME = {"layered": "layered_1024x384", "ragged": "ragged_1024x384", "offset": "offset_2048x768"}
# grid tag of the committed counter summaries, per workload
PMC_TAG = {"layered": "layered_1024x384", "offset": "layered_2048x768"}


def measured_traffic(kname, chosen, workload):
    """HBM bytes per launch of `kname` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE/WRITE_SIZE, scaled by a 1 GiB copy),
    or None when there is none, or it was taken on other kernel source or
    with other settings of the reverse launches (the forward settings leave
    that kernel's bytes alone)."""
    if workload not in PMC_TAG:
        return None
    path = os.path.join(ROOT, "profiles", f"{kname}_pmc_{PMC_TAG[workload]}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        p = json.load(fh)
    if p.get("kernel_source_sha") != kernel_hash():
        return None
    keys = ("graph_steps", "prefetch_reverse", "shots_in_flight_reverse", "tile_rows_reverse",
            "reverse_steps", "graph_branches")
    # the summary's main run and the other reverse launch settings it measured
    for run in [p] + p.get("other_reverse_settings", []):
        if all(run["launch_config"].get(k) == chosen.get(k) for k in keys):
            return run.get("bytes_per_launch")
    return None


def host_cpu():
    """CPU model and the number of cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


_WORKER_WORKLOADS = {}


def _init_oracle_worker(names):
    """Builds the workloads once per worker process, outside the timed work."""
    import oracle  # noqa: F401
    from paper_1406_1864_amd.synthetic import WORKLOADS
    for name in names:
        _WORKER_WORKLOADS[name] = WORKLOADS[name]()


def _oracle_shot_sample(job):
    """One task of the CPU baseline: the FP64 oracle's gradient of shot `s`
    of workload `name` over the first `nsteps` time steps (the whole record
    when nsteps >= its length).  Returns (seconds, steps timed, record length)."""
    name, s, nsteps = job
    import oracle
    from paper_1406_1864_amd.synthetic import Grid
    w = _WORKER_WORKLOADS[name]
    nt_full = int(w.geom.nt[s])
    n = min(nsteps, nt_full)
    geom = w.geom.subset([s]).with_nt(n)
    grid = Grid(w.grid.nz, w.grid.nx, w.grid.dx, w.grid.dt, n, w.grid.nsponge, w.grid.v_ref)
    d_obs = np.zeros((geom.ntrace, n), np.float32)
    t0 = time.perf_counter()
    oracle.gradient(w.v_start, grid, geom, w.wavelet[:n], d_obs, "int")
    return time.perf_counter() - t0, n, nt_full


def oracle_pool(wname, nworkers, nshot):
    """The CPU baseline's process pool, started before this process touches
    the GPU (its workers build the workloads meanwhile)."""
    import multiprocessing as mp
    _, avail = host_cpu()
    P = max(1, min(nworkers or avail, avail, 16, nshot))
    return mp.get_context("spawn").Pool(P, initializer=_init_oracle_worker, initargs=((wname, "anomaly_200x100"),)), P


def cpu_baseline(w, wname, nsteps, pool, P):
    """The FP64 oracle as it stands, timed on the host's cores: a process
    pool with one shot of the workload per worker, each over the first
    `nsteps` time steps (its cost per step is constant: forward sweep with
    snapshots, segment recomputation and adjoint sweep), extrapolated to the
    whole record; beside it the 200x100 anomaly workload (one shot, nt 1000)
    in full on every worker."""
    model, avail = host_cpu()
    with pool:
        pool.map(_oracle_shot_sample, [("anomaly_200x100", 0, 2)] * P, chunksize=1)   # workers up
        t0 = time.perf_counter()
        res = pool.map(_oracle_shot_sample, [(wname, s, nsteps) for s in range(P)], chunksize=1)
        wall = time.perf_counter() - t0
        t1 = time.perf_counter()
        small = pool.map(_oracle_shot_sample, [("anomaly_200x100", 0, 1000)] * P, chunksize=1)
        wall_small = time.perf_counter() - t1
    Z, X = w.grid.padded
    shot_fraction = sum((n - 1) / (nt - 1) for _, n, nt in res)
    cell_steps = sum(3.0 * Z * X * (n - 1) for _, n, _ in res)
    from paper_1406_1864_amd.synthetic import anomaly_200x100
    a = anomaly_200x100()
    Za, Xa = a.grid.padded
    return {"value": shot_fraction / wall, "unit": "shot-gradients/s", "cores": P, "kind": "oracle",
            "gcell_updates_per_s": cell_steps / wall / 1e9, "seconds": wall, "cpu_model": model,
            "cores_available": avail,
            "sample": f"{P} worker processes, one shot each ({wname} shots 0..{P - 1}), the first "
                      f"{res[0][1]} of {res[0][2]} time steps of each (FP64 NumPy, one thread per worker), "
                      f"shot-gradients extrapolated linearly to the whole record",
            "anomaly_200x100_full": {"value": P / wall_small, "unit": "shot-gradients/s", "seconds": wall_small,
                                     "gcell_updates_per_s": P * 3.0 * Za * Xa * 999 / wall_small / 1e9,
                                     "sample": f"{P} workers, each the whole 1-shot, nt 1000 gradient"}}


def time_extended_image(args, grid, geom, w, d_obs, ex, dev):
    """fwi_extended_image against fwi_gradient on the same workload and launch
    configuration: calls per second and the cost of the extra offset sums."""
    import torch
    from paper_1406_1864_amd import binding as B
    H = args.ext
    ws_g = B.workspace(grid, geom, B.WS_GRADIENT, ex, device=dev)
    ws_e = B.workspace(grid, geom, B.WS_EXTIMAGE, ex, H, device=dev)
    res = {}
    for name, fn in (("gradient", lambda: B.gradient(w.v_start, w.wavelet, grid, geom, d_obs, "int", ex,
                                                      illum=False, ws=ws_g, device=dev)),
                     ("extended_image", lambda: B.extended_image(w.v_start, w.wavelet, grid, geom, d_obs, H, "int",
                                                                 ex, ws=ws_e, device=dev))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / args.steps
    nt = geom.nt.astype(np.int64)
    # extra traffic per model cell-step: lam and D written to and read back from
    # the window ring (16 B); the offset sums add (2H+1) x 8 B per cell per window
    return {"hmax": H, "value": geom.nshot / res["extended_image"], "unit": "shot-images/s",
            "ms_per_call": 1e3 * res["extended_image"], "gradient_ms_per_call": 1e3 * res["gradient"],
            "overhead_vs_gradient": res["extended_image"] / res["gradient"] - 1.0,
            "model_cell_steps_per_s": float(np.sum(nt - 1)) * grid.nz * grid.nx / res["extended_image"]}


def time_gn_hvp(args, grid, geom, w, d_obs, ex, dev):
    """fwi_gn_hvp against fwi_gradient on the same workload and launch
    configuration (the product adds the Born field to the forward sweep)."""
    import torch
    from paper_1406_1864_amd import binding as B
    from paper_1406_1864_amd.synthetic import bump_direction
    dv = torch.tensor(bump_direction(grid.nz, grid.nx) * 50.0, dtype=torch.float32, device=dev)
    ws_g = B.workspace(grid, geom, B.WS_GRADIENT, ex, device=dev)
    ws_h = B.workspace(grid, geom, B.WS_GNHVP, ex, device=dev)
    res = {}
    for name, fn in (("gradient", lambda: B.gradient(w.v_start, w.wavelet, grid, geom, d_obs, "int", ex,
                                                      illum=False, ws=ws_g, device=dev)),
                     ("gn_hvp", lambda: B.gn_hvp(w.v_start, w.wavelet, grid, geom, dv, "int", ex, ws=ws_h,
                                                 device=dev))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / args.steps
    return {"value": geom.nshot / res["gn_hvp"], "unit": "shot-products/s", "ms_per_call": 1e3 * res["gn_hvp"],
            "gradient_ms_per_call": 1e3 * res["gradient"],
            "overhead_vs_gradient": res["gn_hvp"] / res["gradient"] - 1.0}


FP32_MFMA_PEAK_TFS = 157.3


def time_offset_diag_exact(args, grid, geom, w, dev, full_shots):
    """fwi_offset_diag_exact on a subset: the first shots and an evenly spread
    subset of their receivers (one group), band up to 4 f_peak, |h| <= 16,
    --exact-sif runs in flight, with the DFT arithmetic(s) of --exact-dft
    (the untimed first call only with --warmup > 0).  Each run (a
    receiver's impulse response or a shot) is a forward sweep that captures
    the model cells' series 8192 / runs-in-flight updates at a time, each
    chunk folded into the run's spectra on the matrix cores (k_dft)."""
    import torch
    from paper_1406_1864_amd import binding as B
    from paper_1406_1864_amd.synthetic import Geometry
    ns = min(args.exact_shots, geom.nshot)
    a, b = int(geom.rec_ptr[0]), int(geom.rec_ptr[1])
    keep = np.linspace(a, b - 1, min(args.exact_diag, b - a)).round().astype(np.int64)
    sub = Geometry(geom.src_iz[:ns].copy(), geom.src_ix[:ns].copy(),
                   (np.arange(ns + 1) * len(keep)).astype(np.int32),
                   np.tile(geom.rec_iz[keep], ns), np.tile(geom.rec_ix[keep], ns), geom.nt[:ns].copy())
    hmax, fmax = 16, 4.0 * w.f_peak
    Z, X = grid.padded
    # runs in flight: the library's default (fwi.h) unless given
    sif = args.exact_sif or (4 if Z * X >= 1_500_000 else 8)
    ex = B.make_exec(shots_in_flight=sif)
    runs = ns + len(keep)
    nt = int(sub.nt[0])
    L = 2 * nt
    K = min(L // 2 + 1, int(np.floor(fmax * L * grid.dt + 1e-9)) + 1)
    model = grid.nz * grid.nx
    dft_flop = 2.0 * model * (nt - 1) * 2 * K           # per run, FP32-equivalent
    chunk = min(nt - 1, max(64, 8192 // min(sif, runs) // 64 * 64))
    full_runs = full_shots + (b - a)
    out = {"unit": "runs/s (forward sweep with series capture + DFT on the matrix cores)", "shots": ns,
           "receivers": int(len(keep)), "hmax": hmax, "fmax_hz": fmax, "bins": K, "nt": nt, "runs_in_flight": sif, "chunk": chunk,
           "dft_shape_per_run": [model, 2 * K, nt - 1], "dft_tflop_per_run": dft_flop / 1e12,
           "cell_updates_per_run": float(Z * X * (nt - 1)), "full_problem_runs": full_runs}
    Dref = D = None
    modes = [m for m in (("fp32", B.DFT_FP32), ("bf16x3", B.DFT_BF16X3)) if args.exact_dft in ("both", m[0])]
    for name, dft in modes:
        print(f"# exact offset diagonal, {name}: {runs} runs", file=sys.stderr, flush=True)
        nbytes = B.fwi_offset_diag_exact_workspace_bytes(grid, sub, ex, hmax, fmax, dft)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        fn = lambda: B.offset_diag_exact(w.v_start, w.wavelet, grid, sub, hmax, fmax, ex, ws=ws, device=dev,
                                         dft=dft)
        if args.warmup > 0:                 # untimed first call
            D = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            D = fn()
        torch.cuda.synchronize()
        call = (time.perf_counter() - t0) / args.steps
        assert bool(torch.isfinite(D).all())
        r = {"value": runs / call, "ms_per_call": 1e3 * call, "ms_per_run": 1e3 * call / runs,
             "workspace_gb": nbytes / 1e9, "full_problem_s_extrapolated": full_runs * call / runs}
        if Dref is None:
            Dref = D.double()
        else:
            r["rel_l2_vs_fp32"] = float(torch.linalg.norm(D.double() - Dref) / torch.linalg.norm(Dref))
        out[name] = r
        del ws
        torch.cuda.empty_cache()
    out["value"] = out[modes[-1][0]]["value"]
    # the aperture-factor reading of the same diagonal (fwi_hessian_diag), its
    # cost and how closely it follows the exact receiver term
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = B.hessian_diag(w.v_start, w.wavelet, grid, sub, B.HESS_OFFSET, hmax, "pm", device=dev)
    torch.cuda.synchronize()
    pa, pb = P.double().flatten(), D.double().flatten()
    am, bm = pa - pa.mean(), pb - pb.mean()
    scale = float(pa @ pb / (pa @ pa))
    out["aperture_factor_reading"] = {
        "seconds": time.perf_counter() - t0,
        "correlation_with_exact": float(am @ bm / (am.norm() * bm.norm())),
        "rel_l2_gap_after_scaling": float((scale * pa - pb).norm() / pb.norm())}
    del D, Dref, P
    torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_offset_diag_exact(w, grid, sub, fmax)
    return out


def cpu_baseline_offset_diag_exact(w, grid, geom, fmax, nsteps=48, ncells=4096):
    """The FP64 oracle's cost of one run of the exact offset diagonal, on a
    bounded sample: its impulse-response modelling (green_series) over the
    first `nsteps` updates of the full grid, and its L-point spectra (power)
    of `ncells` full-length series; both extrapolated linearly to a whole run
    (every update, every model cell)."""
    import oracle
    from paper_1406_1864_amd.synthetic import Grid
    nt = int(geom.nt[0])
    g = Grid(grid.nz, grid.nx, grid.dx, grid.dt, nsteps, grid.nsponge, grid.v_ref)
    t0 = time.perf_counter()
    oracle.green_series(w.v_start, g, int(geom.rec_iz[0]), int(geom.rec_ix[0]), nsteps)
    t_fwd = time.perf_counter() - t0
    L, K, _ = oracle.spectral_bins(nt, grid.dt, fmax)
    x = np.random.default_rng(0).standard_normal((nt - 1, ncells))
    t0 = time.perf_counter()
    oracle.power(x, L, K)
    t_dft = time.perf_counter() - t0
    per_run = t_fwd * (nt - 1) / (nsteps - 1) + t_dft * (grid.nz * grid.nx) / ncells
    return {"value": 1.0 / per_run, "unit": "runs/s", "cores": 1, "kind": "oracle",
            "seconds": t_fwd + t_dft,
            "sample": f"green_series over the first {nsteps} of {nt} updates of the full grid and power() of "
                      f"{ncells} of {grid.nz * grid.nx} cells' {nt - 1}-sample series (FP64 NumPy, single "
                      f"thread), extrapolated linearly to one whole run"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the path would shard by shots "
              "(a subset per GPU and one all-reduce of g, H1, D and J), which is not implemented", file=sys.stderr)
        sys.exit(2)
    pool = npool = None
    if not args.no_cpu:
        pool, npool = oracle_pool(WNAME[args.workload], args.cpu_workers, 32)
    import torch
    from paper_1406_1864_amd import binding as B
    from paper_1406_1864_amd.autograd import FWIProblem, fwi_misfit
    from paper_1406_1864_amd.synthetic import layered_1024x384, offset_2048x768, ragged_1024x384

    dev = "cuda:0"
    torch.cuda.set_device(0)
    B.load()
    # a plain 1 GiB device-to-device copy: reference for the HBM counters and
    # the practically reachable streaming bandwidth on this GPU
    ca = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    cb = torch.empty_like(ca)
    ca.fill_(1.0)
    cb.copy_(ca)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * ca.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb

    make, HM, PK = {"layered": (layered_1024x384, 16, B.PRECOND_SHOT),
                    "ragged": (ragged_1024x384, None, B.PRECOND_SHOT),
                    "offset": (offset_2048x768, 16, B.PRECOND_OFFSET)}[args.workload]
    w = make()
    full_shots = w.geom.nshot
    if args.shots and args.shots != w.geom.nshot:
        w.geom = w.geom.subset(range(args.shots))
    if args.nt:
        from paper_1406_1864_amd.synthetic import Grid
        w.geom = w.geom.with_nt(args.nt)
        w.grid = Grid(w.grid.nz, w.grid.nx, w.grid.dx, w.grid.dt, args.nt, w.grid.nsponge, w.grid.v_ref)
        w.wavelet = w.wavelet[:args.nt]
    grid, geom = w.grid, w.geom
    print(f"# workload {w.name}: {geom.nshot} shots, grid {grid.nz}x{grid.nx}, nt {grid.nt_max}", file=sys.stderr,
          flush=True)

    # recorded data: modelled from the true model with the same engine
    d_obs = B.forward(w.v_true, w.wavelet, grid, geom, B.make_exec(), device=dev)
    torch.cuda.synchronize()
    print("# recorded data modelled", file=sys.stderr, flush=True)
    if args.exec:
        vals = [int(x) for x in args.exec.split(",")]
        S_, TZ_, G_, PF_, PR_ = vals[:5]
        SR_, TZR_, RS_, FS_, GB_ = (vals[5:10] + [0, 0, 0, 0, 0])[:5]
        ex = B.make_exec(shots_in_flight=S_, tile_rows=TZ_, graph_steps=G_, prefetch=PF_, prefetch_reverse=PR_,
                         shots_in_flight_reverse=SR_, tile_rows_reverse=TZR_, reverse_steps=RS_, forward_steps=FS_,
                         graph_branches=GB_)
    else:
        ex = B.make_exec(autotune=1)
    pr = FWIProblem(grid, geom, w.wavelet, d_obs, "int", ex, illum=True, hmax=HM, device=dev)
    v = torch.tensor(w.v_start, device=dev, requires_grad=True)

    def precond(vd, g, problem):
        if PK == B.PRECOND_OFFSET:
            return B.precondition(vd, g, problem.offset, grid, B.PRECOND_OFFSET, hmax=HM, device=dev)
        return B.precondition(vd, g, problem.illum, grid, B.PRECOND_SHOT, device=dev)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    phase = np.zeros(3)

    def step(timed):
        v.grad = None
        if timed:
            ev[0].record()
        J = fwi_misfit(v, pr)
        if timed:
            ev[1].record()
        J.backward()
        if timed:
            ev[2].record()
        gp = precond(v.detach(), v.grad, pr)
        if timed:
            ev[3].record()
            torch.cuda.synchronize()
            phase[0] += ev[0].elapsed_time(ev[1])
            phase[1] += ev[1].elapsed_time(ev[2])
            phase[2] += ev[2].elapsed_time(ev[3])
        return J, gp

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    print("# warmup done; launch configuration:", B.fwi_exec_query(grid, pr.geom, ex, B.WS_AUTOGRAD),
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        J, gp = step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    assert torch.isfinite(J).item() and bool(torch.isfinite(gp).all())

    Z, X = grid.padded
    nt = geom.nt.astype(np.int64)
    shots = geom.nshot
    cell_updates = float(np.sum(3 * Z * X * nt))
    value = shots / (wall / args.steps)
    nrec = np.diff(geom.rec_ptr)
    rev_bytes = float(sum((nt[s] - 1) * reverse_bytes_per_shot_step(grid, int(nrec[s])) for s in range(shots)))
    rev_ms = phase[1] / args.steps
    chosen = B.fwi_exec_query(grid, pr.geom, ex, B.WS_AUTOGRAD)
    # reverse launches per backward: the autograd pair keeps every shot's
    # checkpoints, and its reverse sweep takes the shots (longest records
    # first) `shots_in_flight_reverse` at a time, each group for its longest
    # record, `reverse_steps` time steps per launch
    Sr = max(1, chosen["shots_in_flight_reverse"])
    order = sorted(range(shots), key=lambda s: -int(nt[s]))
    RS = max(1, chosen["reverse_steps"])
    launches = sum((int(nt[order[i0]]) - 1 + RS - 1) // RS for i0 in range(0, shots, Sr))
    launch_us = rev_ms * 1e3 / max(launches, 1)
    bytes_per_launch = rev_bytes / max(launches, 1)
    achieved = bytes_per_launch / (launch_us * 1e-6) / 1e9
    fwd_K = int(np.ceil(np.sqrt(nt.max())))
    fwd_bytes = float(sum((nt[s] - 1) * forward_bytes_per_shot_step(grid, int(nrec[s]), fwd_K)
                          for s in range(shots)))
    full = (shots == full_shots and not args.nt)
    # the dominant kernel: the one-step or the two-step reverse sweep
    rev_kernel = "k_reverse2" if RS == 2 else "k_reverse"
    traffic = measured_traffic(rev_kernel, chosen, args.workload) if full else None
    nrec_mean = float(np.mean(nrec)) if shots else 0.0
    out = {
        "metric": "shot-gradients/s and Gcell-updates/s (fraction of HBM roofline), batched vs plain",
        "value": value,
        "unit": "shot-gradients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name if full else f"{w.name} ({shots} shots, nt {grid.nt_max})",
                   "shots": shots,
                   "grid": [grid.nz, grid.nx], "padded": [Z, X], "nt": int(nt.max()), "receivers_per_shot": nrec_mean,
                   "misfit": "time_integral", "hmax": HM, "path": "autograd, batched, hipGraph, autotuned",
                   "shots_in_flight": chosen["shots_in_flight"], "tile_rows": chosen["tile_rows"],
                   "graph_steps": chosen["graph_steps"], "prefetch": chosen["prefetch"],
                   "prefetch_reverse": chosen["prefetch_reverse"],
                   "shots_in_flight_reverse": chosen["shots_in_flight_reverse"],
                   "tile_rows_reverse": chosen["tile_rows_reverse"],
                   "reverse_steps": chosen["reverse_steps"], "forward_steps": chosen["forward_steps"],
                   "graph_branches": chosen["graph_branches"]},
        "gcell_updates_per_s": cell_updates / (wall / args.steps) / 1e9,
        "phase_ms": {"forward_and_misfit": phase[0] / args.steps, "backward": rev_ms,
                     "precondition": phase[2] / args.steps},
        "roofline": {"bound": "hbm", "kernel": rev_kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_launch, "launches": launches,
                     "avg_launch_us": launch_us,
                     # per padded cell and time step of one shot, and the measured rate
                     "algorithmic_bytes_per_cell_step": bytes_per_launch / (Sr * RS * Z * X),
                     "measured_bytes_per_cell_step": traffic / (Sr * RS * Z * X) if traffic else None,
                     "measured_GBps": traffic / (launch_us * 1e-6) / 1e9 if traffic else None},
        "copy_GBps": copy_gbs,
        "forward_roofline": {"achieved": fwd_bytes / (phase[0] / args.steps * 1e-3) / 1e9, "unit": "GB/s",
                             "frac": fwd_bytes / (phase[0] / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }

    if not args.no_plain:
        ps = min(args.plain_shots, shots)
        pgeom = geom.subset(range(ps))
        pd = d_obs[:pgeom.ntrace].contiguous()
        ppr = FWIProblem(grid, pgeom, w.wavelet, pd, "int", B.make_exec(mode=B.EXEC_PLAIN), illum=True, hmax=HM,
                         device=dev)
        vp = torch.tensor(w.v_start, device=dev, requires_grad=True)

        def pstep():
            vp.grad = None
            Jp = fwi_misfit(vp, ppr)
            Jp.backward()
            return precond(vp.detach(), vp.grad, ppr)

        pstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pstep()
        torch.cuda.synchronize()
        pt = time.perf_counter() - t0
        out["plain"] = {"value": ps / pt, "unit": "shot-gradients/s", "shots": ps,
                        "path": "one shot per launch, one launch per time step, no graph"}
        out["speedup_vs_plain"] = value / (ps / pt)

    if args.ext >= 0:
        out["extended_image"] = time_extended_image(args, grid, geom, w, d_obs, ex, dev)
    if args.gn:
        out["gn_hvp"] = time_gn_hvp(args, grid, geom, w, d_obs, ex, dev)
    if args.exact_diag > 0:
        out["offset_diag_exact"] = time_offset_diag_exact(args, grid, geom, w, dev, full_shots)

    if not args.no_cpu:
        Zc, Xc = w.grid.padded
        # about 15 s per worker: with one worker per core the oracle's gradient costs ~110 ns per
        # padded cell and step (~35 ns on a lone core: the workers share the memory bandwidth)
        nsteps = args.cpu_steps or int(np.clip(15.0 / (Zc * Xc * 1.1e-7), 50, int(w.geom.nt[0])))
        out["cpu_baseline"] = cpu_baseline(w, WNAME[args.workload], nsteps, pool, npool)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
