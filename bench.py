"""Benchmark: ray-cell steps per second of the ERMC radiative heat source on one MI355X, and
the wall time to 1 % RMS error of the learned ray allocation against the plain one.

One step = one full pass of the hot path on one synthetic snapshot whose fields are already
resident in HBM: ingest of the temperature and mole-fraction fields, T_max spectral pdf,
property fields, ray allocation and bucketing, march, per-cell reduction (FP64).

Default workload: the DNS-size snapshot -- 256 x 128 x 128 cells on the 4 pi x 2 x 2 pi box
with tanh-stretched y (gamma 2), periodic x/z, black walls at 300 K, T = 600 + 400 (1 - y^2) K
with 64 Fourier modes of 10 %, H2O and CO2 at 0.1 each with independent +-20 % fluctuations,
seeded synthetic correlated-k tables with 100 bands x 16 g-points rounded to BF16, 64 rays per
cell, FP32 march (double ray geometry and intensity differences), FP64 per-cell sums.
`--workload channel64` runs the 64^3 non-grey channel instead.

Prints one JSON line.  The roofline is that of the dominant kernel, the lane march
(k_march_lane): its duration is the HIP-event time the library records around its launch on
the compute stream, summed over the timed steps; its algorithmic bytes count the steps it
takes (all steps minus those of the long-ray kernel, which the library counts) at 8 bytes per
ray-cell step (an FP32 kappa_{n,g} and an FP32 I_n value of the cell) plus 12 bytes per ray
(an 8-byte work item and a 4-byte ray value).  The kernel itself gathers one 16-byte cell
record per step (the FP64 table coordinate of the temperature and the mole fractions, from
which it interpolates kappa_{n,g} and I_n in LDS tables) and moves 16-byte items and 8-byte
slots; that figure is reported beside.
The `learned` block evaluates the allocation network committed with the package against the
plain allocation on held-out fields of the same generator.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of the march: per ray-cell step one FP32 kappa_{n,g} and one FP32 I_n
# value of the cell; per ray an 8-byte work item and a 4-byte ray value
BYTES_PER_STEP = 4 + 4
BYTES_PER_RAY = 8 + 4
# what the kernel moves: a 16-byte cell record per step, an 8-byte work item and an 8-byte
# slot record {value, steps | end} per ray
KERNEL_BYTES_PER_STEP = 16
KERNEL_BYTES_PER_RAY = 8 + 8
L2_PER_XCD_MB = 4.0
MALL_MB = 256.0
ALLOCATOR_DIR = os.path.join(ROOT, "paper_1810_00188_amd", "allocators")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["dns256", "channel64"], default="dns256",
                    help="throughput workload (default: the DNS-size snapshot)")
    ap.add_argument("--learned-fields", type=int, default=5,
                    help="held-out fields of the learned-vs-plain block of the throughput line (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample (0 disables it)")
    ap.add_argument("--long-ray-steps", type=int, default=0,
                    help="steps a ray takes in the lane kernel before the segmented long-ray "
                         "kernel continues it (0: library default)")
    ap.add_argument("--xcd-span", type=int, default=0,
                    help="consecutive 64-ray chunks each XCD takes in turn (0: library default)")
    ap.add_argument("--alloc-tile", type=int, default=0,
                    help="cells per allocation tile (0: library default, about 1024 tiles)")
    ap.add_argument("--length-sort", type=int, default=-1,
                    help="order of the rays in a bucket: 0 cell order, 1 each march workgroup reorders its "
                         "rays by expected length (-1: library default)")
    ap.add_argument("--bucket-order", type=int, default=0, help="0: longest rays first, 1: band-major")
    ap.add_argument("--region-cells", type=int, default=0,
                    help="cells per region of the march order (0: library default, -1: one region)")
    ap.add_argument("--mg-levels", type=int, default=0,
                    help="multigrid march: grid levels (-1: all the grid allows; 0/1: DNS grid only)")
    ap.add_argument("--mg-steps", type=int, default=0, help="multigrid march: steps per grid (0: 5)")
    ap.add_argument("--mg-study", choices=["channel64", "dns256"], default=None,
                    help="multigrid time and accuracy against the single-grid march, 1..all levels")
    ap.add_argument("--mg-snaps", type=int, default=0, help="snapshots (random streams) per study row")
    ap.add_argument("--batch12", action="store_true",
                    help="12 uneven snapshots (50 bands x 8 g) in one pass: autotuned, eager and HIP graph")
    ap.add_argument("--precision-study", choices=["channel64", "dns256"], default=None,
                    help="errors of the FP32 march and of compensated / plain FP32 sums against FP64")
    ap.add_argument("--learned-cost", choices=["channel64", "dns256"], default=None,
                    help="time of a learned compute (features, network, draws, march) at the workload's R, "
                         "with the committed network or, without one, an untrained one")
    ap.add_argument("--confirm-r1", choices=["channel64", "dns256"], default=None,
                    help="confirm the time to 1 %% RMS error on one held-out field by running the rays per "
                         "cell it predicts, as merged computes of at most --r-max rays, for plain and learned")
    ap.add_argument("--r-max", type=int, default=255, help="rays per cell of one compute in --confirm-r1")
    ap.add_argument("--methods", default="plain,learned", help="--confirm-r1: methods to run (plain, learned)")
    ap.add_argument("--walls-study", action="store_true",
                    help="time per compute with reflecting walls and closed boxes (64^3 workloads)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "reference point that scales rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--learned", choices=["channel64", "dns256"], default=None,
                    help="instead of the throughput benchmark: train the allocation network on plain "
                         "runs and report the wall time to 1 %% RMS error, learned vs plain")
    ap.add_argument("--no-cost", action="store_true",
                    help="train on the second moment alone (no per-(n, g) ray cost in the loss)")
    ap.add_argument("--train-rays", type=int, default=0, help="rays per training cell (0: the workload's R)")
    ap.add_argument("--train-seeds", type=int, default=0, help="training fields (0: per workload)")
    ap.add_argument("--eval-seeds", type=int, default=0, help="held-out evaluation fields (0: per workload)")
    ap.add_argument("--train-steps", type=int, default=0, help="Adam steps (0: per workload)")
    ap.add_argument("--batch-cells", type=int, default=0, help="cells per Adam step (0: per workload)")
    ap.add_argument("--save-allocator", action="store_true",
                    help="store the trained network with the package (allocators/<workload>.npz)")
    ap.add_argument("--mix-eps", type=float, default=0.1,
                    help="weight of the plain pdf mixed into the learned one (defensive mixture)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "march_traffic.json"),
                    help="HBM bytes per march launch measured by rocprofv3 (optional)")
    return ap.parse_args()


def kernel_source_hash():
    """sha256 over the HIP sources (the traffic counters are valid for that code only)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1810_00188_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_baseline(w, target_s, stride=1, stride_1core=16):
    """The oracle, as it stands, on a bounded sample of the same workload: every stride-th cell
    of the grid (all R rays of each) on all host threads, in passes with fresh snapshot numbers
    (fresh random streams) until about target_s seconds have elapsed (at least one), then every
    stride_1core-th cell on one thread for about a quarter of that."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()

    def run(cells, nthreads, budget):
        steps = passes = 0
        t0 = time.perf_counter()
        while True:
            P = oracle.Problem(w.replace(snap=w.snap + 1 + passes))
            _, _, st = oracle.divergence(P, cells=cells, nthreads=nthreads)
            steps += st
            passes += 1
            dt = time.perf_counter() - t0
            if dt >= budget:
                return steps, passes, dt

    cells = None if stride == 1 else np.arange(0, w.ncells, stride)
    nsel = w.ncells if cells is None else len(cells)
    steps, passes, dt = run(cells, threads, target_s)
    what = "whole grid" if stride == 1 else f"every {stride}th cell"
    out = {"value": steps / dt, "unit": "ray-cell steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{passes} pass(es) of the same workload over {what} ({nsel} of {w.ncells} cells x {w.R} "
                     f"rays, all {threads} host threads), {steps} steps in {dt:.1f} s"}
    cells1 = np.arange(0, w.ncells, stride_1core)
    steps1, passes1, dt1 = run(cells1, 1, target_s / 4)
    out["value_1core"] = steps1 / dt1
    out["sample_1core"] = (f"{passes1} pass(es) over every {stride_1core}th cell ({len(cells1)} cells x {w.R} rays) "
                           f"on one thread, {steps1} steps in {dt1:.1f} s")
    return out


def say(msg):
    print(f"[learned] {msg}", flush=True)


def learned_bench(a):
    """Wall time to 1 % RMS error of the heat source, learned vs plain allocation (median over
    held-out fields), with the network trained by the library's kernels on plain runs."""
    import numpy as np
    import torch
    from paper_1810_00188_amd import inputs, learned, rmc

    cfg = {"channel64": dict(gen=inputs.channel64, train=64, eval=20, steps=12000, cells=16384, batch=256,
                             rays=0, Rs=(16, 32, 64, 128)),
           "dns256": dict(gen=inputs.dns256, train=200, eval=20, steps=40000, cells=65536, batch=256,
                          rays=0, Rs=(16, 32, 64, 128))}[a.learned]
    n_train = a.train_seeds or cfg["train"]
    n_eval = a.eval_seeds or cfg["eval"]
    steps = a.train_steps or cfg["steps"]
    eps, lr = a.mix_eps, 2e-3
    t_start = time.perf_counter()
    w0 = cfg["gen"](field_seed=1)
    kd = w0.kd
    nu_c, gx = learned.spectral_inputs(kd)
    s = rmc.Solver(0)
    s.set_workload(w0, device_fields=True, mix_eps=eps)
    rng = np.random.default_rng(7)
    runs, feats = [], []
    for k in range(1, n_train + 1):
        w = w0 if k == 1 else cfg["gen"](field_seed=k)
        s.set_temperature(np.ascontiguousarray(w.T, dtype=np.float32))
        s.set_species(np.ascontiguousarray(w.X, dtype=np.float32))
        s.set_options(rmc.default_options(rays_per_cell=a.train_rays or cfg["rays"] or w.R, seed=w.seed, snapshot=k, tol=w.tol,
                                          max_steps=w.max_steps, march=rmc.F32, mix_eps=eps))
        cells = np.sort(rng.choice(w.ncells, min(cfg["cells"], w.ncells), replace=False))
        runs.append(learned.plain_samples(s, cells))
        feats.append(runs[-1].feat.cpu().numpy())
        say(f"training field {k}: {len(cells)} cells x {s.R} rays")
    mu, sd = learned.standardisation(feats, kd)
    s.set_allocator(learned.init_params(0), mu, sd, nu_c, gx)
    t_train = time.perf_counter()
    batch_cells = a.batch_cells or cfg["batch"]
    losses = learned.train(s, runs, steps, lr, batch_cells, log=say, use_cost=not a.no_cost)
    t_train = time.perf_counter() - t_train
    params = s.get_allocator()
    curve = [float(np.mean(losses[max(0, q - 200):q + 1])) for q in
             sorted(set([min(len(losses) - 1, int(len(losses) * f)) for f in (0.0, 0.05, 0.1, 0.25, 0.5, 0.75, 1.0)]))]
    info = {"workload": a.learned, "train_fields": n_train, "train_field_seeds": [1, n_train],
            "train_cells_per_field": cfg["cells"], "train_rays_per_cell": a.train_rays or cfg["rays"] or w0.R,
            "adam_steps": steps, "batch_cells": batch_cells, "lr": [lr, lr / 10.0], "mix_eps": eps,
            "loss": "second moment" if a.no_cost else "second moment x ray cost",
            "loss_curve_steps_frac": [0.0, 0.05, 0.1, 0.25, 0.5, 0.75, 1.0], "loss_curve": curve,
            "train_s": t_train}
    if a.save_allocator:
        from paper_1810_00188_amd import allocators
        say(f"saved {allocators.save(a.learned, params, mu, sd, eps, info)}")
    del runs
    s.close()
    s_plain = rmc.Solver(0)
    s_learn = rmc.Solver(0)
    results = []
    for e in range(n_eval):
        w = cfg["gen"](field_seed=1000 + e)
        s_plain.set_workload(w, device_fields=True)
        s_learn.set_workload(w, device_fields=True, sampling=rmc.SAMPLING_LEARNED, mix_eps=eps)
        s_learn.set_allocator(params, mu, sd, nu_c, gx)
        say(f"evaluation field {1000 + e}")
        results.append(learned.time_to_error(w, s_plain, s_learn, eps, Rs=cfg["Rs"], log=say, alloc_cache=1))
    tp = np.array([r["plain"]["time_to_target_merged_s"] for r in results])
    tl = np.array([r["learned"]["time_to_target_merged_s"] for r in results])
    tp1 = np.array([r["plain"]["time_to_target_s"] for r in results])
    tl1 = np.array([r["learned"]["time_to_target_s"] for r in results])
    out = {
        "metric": "wall time to 1% RMS divq error, learned vs plain (computes of 255 rays per cell: "
                  "ceil(R_1% / 255) (t0 + 255 t1))",
        "value": float(np.median(tl)), "unit": "s", "higher_is_better": False,
        "plain_s": float(np.median(tp)), "speedup_vs_plain": float(np.median(tp / tl)),
        "learned_wins": int(np.sum(tl < tp)), "eval_fields": n_eval,
        "single_compute_model": {"learned_s": float(np.median(tl1)), "plain_s": float(np.median(tp1)),
                                 "speedup_vs_plain": float(np.median(tp1 / tl1)), "learned_wins": int(np.sum(tl1 < tp1)),
                                 "note": "t0 + t1 R_1%, as if one compute carried all R_1% rays per cell"},
        "n_gpus": 1, "dtype": "f32", "data": "synthetic", "vs_baseline": None,
        "config": {"workload": w0.name, "grid": [w0.nx, w0.ny, w0.nz], "bands": kd.nb, "g_points": kd.ng,
                   "train_fields": n_train, "train_cells_per_field": cfg["cells"], "train_steps": steps,
                   "train_rays_per_cell": a.train_rays or cfg["rays"] or w0.R,
                   "batch_cells": batch_cells, "mix_eps": eps, "R": list(cfg["Rs"]),
                   "loss": "second moment" if a.no_cost else "second moment x ray cost",
                   "reference_rays_per_cell": results[0]["ref_rays_per_cell"]},
        "train_loss_first_last": [float(np.mean(losses[:50])), float(np.mean(losses[-50:]))],
        "train_loss_curve": curve,
        "train_s": t_train, "total_s": time.perf_counter() - t_start,
        "per_field": [{"plain": r["plain"], "learned": r["learned"]} for r in results],
    }
    print(json.dumps(out), flush=True)


def grid_levels(nx, ny, nz):
    """Grid levels the multigrid march can use (coarsening ratio 2, axes even, halves >= 3)."""
    L = 1
    while L < 8 and all(n % 2 == 0 and n // 2 >= 3 for n in (nx, ny, nz)):
        nx, ny, nz = nx // 2, ny // 2, nz // 2
        L += 1
    return L


def mg_study(a):
    """Multigrid march (Sec. 4.3) against the single-grid march on one field: wall time per
    compute and speedup for 1 .. all grid levels (5 steps per grid, then 10 and 20 on all
    levels), and the accuracy of the estimate.  Every row uses the same seeds, so the rays
    (band, g, octant, direction) are the same and the difference of the estimates is the
    multigrid approximation plus a small residue of noise; it is averaged over several
    snapshots (random streams) and compared with the Monte Carlo standard error of one
    compute."""
    import numpy as np
    import torch
    from paper_1810_00188_amd import inputs, rmc

    gen = {"channel64": inputs.channel64, "dns256": inputs.dns256}[a.mg_study]
    w = gen()
    nmax = grid_levels(w.nx, w.ny, w.nz)
    K = a.mg_snaps or (8 if a.mg_study == "channel64" else 3)
    dev = torch.device("cuda", 0)
    s = rmc.Solver(0)
    s.set_workload(w, device_fields=True)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device=dev)
    se = torch.zeros_like(dq)
    rows_cfg = [(1, 5)] + [(L, 5) for L in range(2, nmax + 1)] + [(nmax, 10), (nmax, 20)]
    rows, base = [], None
    for L, S in rows_cfg:
        def opts(k):
            return rmc.default_options(rays_per_cell=w.R, seed=w.seed, snapshot=100 + k, tol=w.tol,
                                       max_steps=w.max_steps, march=rmc.F32, accum=rmc.ACC[w.accum],
                                       mg_levels=L, mg_steps=S)
        s.set_options(opts(0))
        for _ in range(2):
            s.compute(dq, se)
        torch.cuda.synchronize()
        qs, ses, t_tot, steps, march = [], [], 0.0, 0, 0.0
        for k in range(K):
            s.set_options(opts(k))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.compute(dq, se)
            torch.cuda.synchronize()
            t_tot += time.perf_counter() - t0
            st = s.stats()
            steps += st["steps"]
            march += st["ms_march"]
            qs.append(dq.cpu().numpy())
            ses.append(se.cpu().numpy())
        q = np.mean(qs, axis=0)
        se_rms = float(np.sqrt(np.mean(np.square(ses))))
        row = {"levels": L, "steps_per_grid": S, "ms_per_compute": 1e3 * t_tot / K, "march_ms": march / K,
               "steps_per_ray": steps / (K * w.ncells * w.R)}
        if base is None:
            base = dict(q=q, ms=row["ms_per_compute"], se=se_rms)
        rms_q = float(np.sqrt(np.mean(base["q"] ** 2)))
        row["speedup"] = base["ms"] / row["ms_per_compute"]
        row["rms_diff_vs_single_rel"] = float(np.sqrt(np.mean((q - base["q"]) ** 2))) / rms_q
        row["mean_diff_vs_single_rel"] = float(np.mean(q - base["q"])) / rms_q
        row["stderr_one_compute_rel"] = se_rms / rms_q
        row["stderr_ratio_vs_single"] = se_rms / base["se"]
        rows.append(row)
        print(f"[mg] {json.dumps(row)}", flush=True)
    out = {"metric": "multigrid march: time per compute and accuracy vs the single-grid march",
           "unit": "ms", "n_gpus": 1, "dtype": "f32", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "bands": w.kd.nb, "g_points": w.kd.ng,
                      "rays_per_cell": w.R, "snapshots_per_row": K, "grid_levels_allowed": nmax},
           "rows": rows}
    print(json.dumps(out), flush=True)
    s.close()


def precision_study(a):
    """Errors of the reduced-precision paths against FP64 on one field, same seeds (so the
    same rays: band, g, octant and direction are drawn in FP64 either way):
    - ray values of the FP32 march against the FP64 march (sampled cells, all their rays),
      with the share of rays whose step count differs (tau crossing tol within rounding);
    - cell estimates of the FP32 march against the FP64 march (FP64 sums on both sides);
    - per-cell sums of the FP32 march's rays in compensated FP32 and in plain FP32 against
      FP64 sums of the same rays.
    Errors are stated relative to the RMS of the FP64 quantity and, for cell estimates, to
    the Monte Carlo standard error of the compute."""
    import numpy as np
    import torch
    from paper_1810_00188_amd import inputs, rmc

    gen = {"channel64": inputs.channel64, "dns256": inputs.dns256}[a.precision_study]
    w = gen()
    dev = torch.device("cuda", 0)
    s = rmc.Solver(0)
    s.set_workload(w, device_fields=True)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device=dev)
    se = torch.zeros_like(dq)
    stride = 1 if w.ncells <= 262144 else 16
    cells = np.arange(0, w.ncells, stride)

    def run(march, accum):
        s.set_options(rmc.default_options(rays_per_cell=w.R, seed=w.seed, snapshot=w.snap, tol=w.tol,
                                          max_steps=w.max_steps, march=march, accum=rmc.ACC[accum]))
        s.compute(dq, se)
        torch.cuda.synchronize()
        return dq.cpu().numpy().copy(), se.cpu().numpy().copy()

    q64, se64 = run(rmc.F64, "f64")
    Y64, S64 = s.ray_values(cells)
    q32, se32 = run(rmc.F32, "f64")
    Y32, S32 = s.ray_values(cells)
    qc, _ = run(rmc.F32, "comp32")
    qf, _ = run(rmc.F32, "f32")
    rms = lambda v: float(np.sqrt(np.mean(np.square(v))))  # noqa: E731
    dY = Y32 - Y64
    same = S32 == S64
    rmsY, rmsQ, rms_se = rms(Y64), rms(q64), rms(se64)
    out = {"metric": "errors of reduced precision against FP64", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "bands": w.kd.nb, "g_points": w.kd.ng,
                      "rays_per_cell": w.R, "ray_sample": f"every {stride}th cell, all its rays ({Y64.size} rays)"},
           "ray_fp32_march_vs_fp64": {
               "max_abs_over_rms": float(np.abs(dY).max()) / rmsY,
               "rms_over_rms": rms(dY) / rmsY,
               "max_abs_over_rms_same_steps": float(np.abs(dY[same]).max()) / rmsY if same.any() else None,
               "rel_err_max_where_abs_Y_above_rms": float((np.abs(dY)[np.abs(Y64) > rmsY] / np.abs(Y64[np.abs(Y64) > rmsY])).max()),
               "rays_with_other_step_count": int((~same).sum()),
               "share_other_step_count": float((~same).mean())},
           "cell_fp32_march_vs_fp64": {
               "max_abs_over_rms": float(np.abs(q32 - q64).max()) / rmsQ,
               "rms_over_rms": rms(q32 - q64) / rmsQ,
               "rms_over_mc_stderr": rms(q32 - q64) / rms_se},
           "cell_sums_comp_fp32_vs_fp64": {
               "max_abs_over_rms": float(np.abs(qc - q32).max()) / rmsQ,
               "rms_over_rms": rms(qc - q32) / rmsQ,
               "max_rel_where_abs_above_rms": float((np.abs(qc - q32)[np.abs(q32) > rmsQ] / np.abs(q32[np.abs(q32) > rmsQ])).max())},
           "cell_sums_plain_fp32_vs_fp64": {
               "max_abs_over_rms": float(np.abs(qf - q32).max()) / rmsQ,
               "rms_over_rms": rms(qf - q32) / rmsQ,
               "max_rel_where_abs_above_rms": float((np.abs(qf - q32)[np.abs(q32) > rmsQ] / np.abs(q32[np.abs(q32) > rmsQ])).max())},
           "mc_stderr_rms_over_rms_q": rms_se / rmsQ}
    print(json.dumps(out), flush=True)
    s.close()


def learned_cost(a):
    """Phase times of a compute with the learned allocation (the allocation network, softmax
    and draws run in the prep phase) beside a plain compute of the same field."""
    import numpy as np
    import torch
    from paper_1810_00188_amd import allocators, inputs, learned, rmc

    gen = {"channel64": inputs.channel64, "dns256": inputs.dns256}[a.learned_cost]
    w = gen(field_seed=1000)
    try:
        net = allocators.load(a.learned_cost)
        params, mu, sd, eps, which = net["params"], net["mu"], net["sd"], net["mix_eps"], "committed network"
    except FileNotFoundError:
        params, which, eps = learned.init_params(0), "untrained network", 0.1
        mu, sd = learned.standardisation([np.zeros((1, 3), np.float32)], w.kd)
        sd[:3] = 1.0
    nu_c, gx = learned.spectral_inputs(w.kd)
    dev = torch.device("cuda", 0)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device=dev)
    rows = {}
    for name, sampling, cache in (("plain", rmc.SAMPLING_PLAIN, 0), ("learned", rmc.SAMPLING_LEARNED, 0),
                                  ("learned, allocation cache", rmc.SAMPLING_LEARNED, 1)):
        s = rmc.Solver(0)
        s.set_workload(w, device_fields=True, sampling=sampling, mix_eps=eps if sampling else 0.0, alloc_cache=cache)
        if sampling:
            s.set_allocator(params, mu, sd, nu_c, gx)
        s.compute(dq)
        torch.cuda.synchronize()
        s.reset_stats()
        K = 3
        t0 = time.perf_counter()
        for _ in range(K):
            s.compute(dq)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / K
        st = s.stats()
        rows[name] = {"ms_per_compute": 1e3 * dt, "prep_ms": st["sum_ms_prep"] / K, "alloc_ms": st["sum_ms_alloc"] / K,
                      "march_ms": st["sum_ms_march"] / K, "reduce_ms": st["sum_ms_reduce"] / K,
                      "steps_per_ray": st["sum_steps"] / (K * w.ncells * w.R)}
        print(f"[learned-cost] {name}: {json.dumps(rows[name])}", flush=True)
        s.close()
    print(json.dumps({"metric": "learned compute phase times", "unit": "ms", "network": which,
                      "config": {"workload": w.name, "rays_per_cell": w.R}, "rows": rows}), flush=True)


def confirm_r1(a):
    """Time to 1 % RMS error confirmed by running it.  On held-out field 1000: the protocol of
    `learned.time_to_error` estimates R_1% (rays per cell for a 1 % error) and t(R) for each
    method; then K = ceil(R_1% / r_max) computes of r_max rays per cell (distinct snapshot
    streams) are enqueued back to back and summed on the device, alternately into halves A and
    B.  The estimate Q averages all K, and the difference of the halves measures its error
    without a reference: Var(Q_A - Q_B) = Var(Q) K^2 / (n_A n_B), so
    e = RMS(Q_A - Q_B) sqrt(n_A n_B) / K / RMS(Q) (RMS(Q_A - Q_B) / (2 RMS(Q)) for even K).
    The wall time of the K computes is the measured time to 1 %."""
    import math
    import numpy as np
    import torch
    from paper_1810_00188_amd import allocators, inputs, learned, rmc

    gen = {"channel64": inputs.channel64, "dns256": inputs.dns256}[a.confirm_r1]
    net = allocators.load(a.confirm_r1)
    w = gen(field_seed=1000)
    nu_c, gx = learned.spectral_inputs(w.kd)
    dev = torch.device("cuda", 0)
    s_plain, s_learn = rmc.Solver(0), rmc.Solver(0)
    s_plain.set_workload(w, device_fields=True)
    s_learn.set_workload(w, device_fields=True, sampling=rmc.SAMPLING_LEARNED, mix_eps=net["mix_eps"])
    s_learn.set_allocator(net["params"], net["mu"], net["sd"], nu_c, gx)
    say = lambda m: print(f"[confirm] {m}", flush=True)  # noqa: E731
    est = learned.time_to_error(w, s_plain, s_learn, net["mix_eps"], Rs=(16, 32, 64, 128), log=say, alloc_cache=1)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device=dev)
    rms = lambda v: float(np.sqrt(np.mean(np.square(v))))  # noqa: E731
    rows = {}
    for name, s, sampling in (("plain", s_plain, rmc.SAMPLING_PLAIN), ("learned", s_learn, rmc.SAMPLING_LEARNED)):
        if name not in a.methods.split(","):
            continue
        R1 = est[name]["R_target"]
        K = max(2, math.ceil(R1 / a.r_max))
        halves = [torch.zeros_like(dq), torch.zeros_like(dq)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(K):
            s.set_options(rmc.default_options(rays_per_cell=a.r_max, seed=w.seed, snapshot=20000 + k, tol=w.tol,
                                              max_steps=w.max_steps, march=rmc.F32, accum=rmc.ACC[w.accum],
                                              sampling=sampling, mix_eps=net["mix_eps"] if sampling else 0.0,
                                              alloc_cache=1 if sampling else 0))
            s.compute(dq)
            halves[k & 1] += dq
            if (k + 1) % max(1, K // 10) == 0:
                torch.cuda.synchronize()
                say(f"{name}: {k + 1} of {K} computes, {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t0
        nA, nB = (K + 1) // 2, K // 2
        qa, qb = (halves[0] / nA).cpu().numpy(), (halves[1] / nB).cpu().numpy()
        q = (nA * qa + nB * qb) / K
        # Var(Q_A - Q_B) = Var(Q) K^2 / (nA nB): scale the half difference to the error of Q
        e = rms(qa - qb) * math.sqrt(nA * nB) / K / rms(q)
        m = est[name]
        rows[name] = {"R_1pct_estimated": R1, "computes": K, "rays_per_cell_per_compute": a.r_max,
                      "rays_per_cell": K * a.r_max, "rel_err_measured": e,
                      "rel_err_expected_at_these_rays": 0.01 * math.sqrt(R1 / (K * a.r_max)),
                      "time_s_measured": t_run,
                      "time_s_fit_single_compute": m["time_to_target_s"],
                      "time_s_fit_merged": m["t_first_s"] + K * (m["t0_s"] + m["t_per_ray_s"] * a.r_max),
                      "t0_s": m["t0_s"], "t_per_ray_s": m["t_per_ray_s"], "err_slope": m["err_slope"],
                      "rel_err_R16_128": m["rel_err"], "t_s_R16_128": m["t_s"]}
        say(f"{name}: {json.dumps(rows[name])}")
    out = {"metric": "wall time to 1% RMS divq error, confirmed by merged computes", "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "field_seed": 1000,
                      "network": net["info"], "r_max": a.r_max},
           "rows": rows}
    if len(rows) == 2:
        out["speedup_vs_plain"] = rows["plain"]["time_s_measured"] / rows["learned"]["time_s_measured"]
    print(json.dumps(out), flush=True)
    s_plain.close()
    s_learn.close()


def walls_study(a):
    """Wall rows (Eq. 3's wall factor with specular reflection, closed boxes of Table 1): time
    per compute, steps per ray and ray-cell steps per second on 64^3 workloads, black walls
    against reflecting ones.  Fields resident on the GPU; 2 warm-up and 5 timed computes."""
    import numpy as np
    import torch
    from paper_1810_00188_amd import inputs, rmc

    cases = [("channel 64^3, black walls (benchmark workload)", inputs.channel64()),
             ("channel 64^3, walls eps = 0.5", inputs.channel64().replace(eps_walls=(0.5, 0.5))),
             ("channel 64^3, walls eps = 0.1", inputs.channel64().replace(eps_walls=(0.1, 0.1))),
             ("cube 64^3 Case 12 field, black walls", inputs.cube_3dimens(64)),
             ("cube 64^3 Case 12 field, walls eps = 0.5", inputs.cube_3dimens(64, eps_walls=0.5)),
             ("cube 64^3 Case 3 (sin field, grey kappa 0.5), black walls, FP32",
              inputs.sin_cube(64, kappa=0.5, R=32).replace(march="f32"))]
    dev = torch.device("cuda", 0)
    rows = []
    for name, w in cases:
        s = rmc.Solver(0)
        s.set_workload(w, device_fields=True)
        dq = torch.zeros(w.ncells, dtype=torch.float64, device=dev)
        for _ in range(2):
            s.compute(dq)
        torch.cuda.synchronize()
        s.reset_stats()
        t0 = time.perf_counter()
        for _ in range(5):
            s.compute(dq)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        st = s.stats()
        row = {"case": name, "ms_per_compute": 1e3 * dt, "march_ms": st["sum_ms_march"] / 5,
               "steps_per_ray": st["sum_steps"] / (5 * w.ncells * w.R), "steps_per_s": st["sum_steps"] / (5 * dt),
               "long_steps_share": st["long_steps"] / max(st["steps"], 1)}
        rows.append(row)
        print(f"[walls] {json.dumps(row)}", flush=True)
        s.close()
    print(json.dumps({"metric": "walls: time per compute and ray-cell steps/s", "unit": "ms", "n_gpus": 1,
                      "dtype": "f32", "data": "synthetic", "vs_baseline": None, "rows": rows}), flush=True)


def batch12_bench(a):
    """The batched configuration: 12 snapshots of uneven size (3 each of 64^3, 96x64x64, 128^3,
    192x96x96; stretched y; 50 bands x 8 g; R = 32; FP32 march, FP64 sums) in one pipeline pass
    -- one bucketing and one march launch over all of them -- with the launch schedule picked by
    the autotuner, timed eagerly (rmc_compute_batch) and as a captured HIP graph replayed."""
    import torch
    from paper_1810_00188_amd import inputs, rmc

    ws = inputs.batch12()
    dev = torch.device("cuda", 0)
    solvers = []
    for w in ws:
        s = rmc.Solver(0)
        s.set_workload(w, device_fields=True)
        solvers.append(s)
    t0 = time.perf_counter()
    choice = rmc.autotune_batch(solvers, reps=1)
    t_tune = time.perf_counter() - t0
    outs = [torch.zeros(w.ncells, dtype=torch.float64, device=dev) for w in ws]
    for _ in range(2):
        rmc.compute_batch(solvers, outs)
    torch.cuda.synchronize()
    solvers[0].reset_stats()
    K = 5
    t0 = time.perf_counter()
    for _ in range(K):
        rmc.compute_batch(solvers, outs)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / K
    st = solvers[0].stats()
    steps, rays = st["steps"], st["rays"]
    cs = torch.cuda.Stream()             # capture needs a stream of its own (default priority)
    with torch.cuda.stream(cs):
        g = rmc.Graph(solvers, outs)
        g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2 * K):
            g.launch()
        torch.cuda.synchronize()
        graph = (time.perf_counter() - t0) / (2 * K)
        g.close()
    out = {"metric": "batched snapshots: ray-cell steps/s", "value": steps / graph, "unit": "ray-cell steps/s",
           "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic", "vs_baseline": None,
           "config": {"workload": "12 snapshots: 3 x 64^3, 3 x 96x64x64, 3 x 128^3, 3 x 192x96x96, stretched y, "
                                  "50 bands x 8 g, 32 rays/cell, FP32 march, FP64 sums",
                      "cells": sum(w.ncells for w in ws), "rays_per_batch": rays, "steps_per_batch": steps},
           "ms_per_batch_graph": 1e3 * graph, "ms_per_batch_eager": 1e3 * eager,
           "steps_per_s_eager": steps / eager, "autotune": choice, "autotune_s": t_tune,
           "phases_ms_eager": {"prep": st["ms_prep"], "alloc": st["ms_alloc"], "march": st["ms_march"],
                               "reduce": st["ms_reduce"]}}
    print(json.dumps(out), flush=True)
    for s in solvers:
        s.close()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.learned:
        learned_bench(a)
        return
    if a.mg_study:
        mg_study(a)
        return
    if a.walls_study:
        walls_study(a)
        return
    if a.precision_study:
        precision_study(a)
        return
    if a.learned_cost:
        learned_cost(a)
        return
    if a.confirm_r1:
        confirm_r1(a)
        return
    if a.batch12:
        batch12_bench(a)
        return
    import torch

    dev = torch.device("cuda", 0)
    if a.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 4, "copies": 3}), flush=True)
        return
    throughput(a)


WORKLOADS = {
    "dns256": ("DNS-size snapshot 256x128x128, tanh-stretched y, 64 modes at 10 %, H2O + CO2 +-20 %, "
               "100 bands x 16 g (BF16-rounded tables), 64 rays/cell, FP32 march, FP64 sums",
               dict(cpu_stride=1, cpu_stride_1core=256)),
    "channel64": ("non-grey channel 64x64x64, 20 bands x 7 g, 32 rays/cell, FP32 march, FP64 sums",
                  dict(cpu_stride=1, cpu_stride_1core=16)),
}


def workload_of(name):
    from paper_1810_00188_amd import inputs
    return {"dns256": inputs.dns256, "channel64": inputs.channel64}[name]()


def traffic_record(path, workload):
    """HBM bytes per k_march_lane launch measured by rocprofv3 for this workload, if the record
    was taken on the current HIP sources (else None)."""
    if not (path and os.path.exists(path)):
        return None
    rec = json.load(open(path)).get("k_march_lane", {}).get(workload)
    if not rec or rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec


def throughput(a):
    import numpy as np
    import torch
    from paper_1810_00188_amd import rmc

    dev = torch.device("cuda", 0)
    desc, wcfg = WORKLOADS[a.workload]
    w = workload_of(a.workload)
    s = rmc.Solver(0)
    overrides = {k: v for k, v in (("long_ray_steps", a.long_ray_steps), ("xcd_span", a.xcd_span),
                                   ("bucket_order", a.bucket_order), ("mg_levels", a.mg_levels),
                                   ("mg_steps", a.mg_steps), ("alloc_tile", a.alloc_tile),
                                   ("region_cells", a.region_cells)) if v}
    if a.length_sort >= 0:
        overrides["length_sort"] = a.length_sort
    mg = a.mg_levels not in (0, 1)
    s.set_workload(w, **overrides)
    T = torch.from_numpy(np.ascontiguousarray(w.T, dtype=np.float32)).to(dev)
    X = torch.from_numpy(np.ascontiguousarray(w.X, dtype=np.float32)).to(dev)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device=dev)
    se = torch.zeros_like(dq)

    def step():
        s.set_fields(T, X)          # ingest of the snapshot's fields (one synchronisation)
        s.compute(dq, se)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    s.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(a.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = s.stats()
    elapsed = t1 - t0
    steps_total = st["sum_steps"]
    assert st["computes"] == a.steps, st
    value = steps_total / elapsed
    march_ms = st["sum_ms_march"] / a.steps
    lane_ms = st["sum_ms_march_lane"] / a.steps
    lane_steps = st["steps"] - st["long_steps"]
    rays = st["rays"]
    bytes_launch = BYTES_PER_STEP * lane_steps + BYTES_PER_RAY * rays
    kbytes_launch = KERNEL_BYTES_PER_STEP * lane_steps + KERNEL_BYTES_PER_RAY * rays
    achieved = bytes_launch / (lane_ms * 1e-3) / 1e9
    rec = None if mg else traffic_record(a.traffic_json, a.workload)
    # the march's access pattern alone (no physics): the gather rate it can reach, in steps/s
    probe_steps = max(1, int(round(lane_steps / max(rays, 1))))
    pms = min(s.gather_probe(probe_steps)[0] for _ in range(3))
    probe_rate = rays * probe_steps / (pms * 1e-3)
    lane_rate = lane_steps / (lane_ms * 1e-3)
    ncpad = 64 * ((w.nx + 3) // 4) * ((w.ny + 3) // 4) * ((w.nz + 3) // 4)
    ws_mb = ncpad * 16 / 1e6           # the cell records, shared by every (band, g) pair
    level = "L2" if ws_mb <= L2_PER_XCD_MB else ("MALL" if ws_mb <= MALL_MB else "HBM")
    out = {
        "metric": "ray-cell steps/s",
        "value": value,
        "unit": "ray-cell steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc + (f", multigrid march {a.mg_levels} levels x {a.mg_steps or 5} steps"
                                       if mg else ""),
                   "grid": [w.nx, w.ny, w.nz], "bands": w.kd.nb, "g_points": w.kd.ng,
                   "rays_per_cell": w.R, "rays_per_step": rays,
                   "ray_cell_steps_per_step": st["steps"], "parallelism": "1 GPU"},
        "phases_ms": {"prep": st["sum_ms_prep"] / a.steps, "alloc": st["sum_ms_alloc"] / a.steps,
                      "march": march_ms, "reduce": st["sum_ms_reduce"] / a.steps},
        "march_steps_per_s": st["steps"] / (march_ms * 1e-3),
        "march_steps_split": {"lane": lane_steps, "long": st["long_steps"]},
        "roofline": {"kernel": "k_march_mg" if mg else "k_march_lane", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": rec["bytes_per_launch"] if rec else None,
                     "ms_per_launch": lane_ms,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "bytes_model": f"{BYTES_PER_STEP} B per ray-cell step + {BYTES_PER_RAY} B per ray",
                     "steps_per_launch": lane_steps, "rays_per_launch": rays,
                     "kernel_bytes_per_launch": kbytes_launch,
                     "kernel_gbs": kbytes_launch / (lane_ms * 1e-3) / 1e9,
                     "working_set_mb": ws_mb, "working_set_level": level,
                     "lane_steps_per_s": lane_rate,
                     "probe_steps_per_s": probe_rate,
                     "frac_of_achievable_steps": lane_rate / probe_rate,
                     "achievable_probe": f"rmc_gather_probe: {rays} lanes x {probe_steps} steps of the "
                                         f"march's access pattern without the physics, {pms:.3f} ms"},
    }
    if rec and "valu_issue" in rec:
        # what the rocprofv3 counters of this kernel (same sources) say binds it
        out["roofline"]["measured_limiter"] = {"valu_issue": rec["valu_issue"], "l2_hit_rate": rec["l2_hit_rate"],
                                               "mall_bytes_per_step": rec["bytes_per_launch"] / lane_steps,
                                               "source": "profiles/march_dns256_traffic.md"}
    s.close()
    del T, X, dq, se
    torch.cuda.empty_cache()
    if a.learned_fields > 0 and not mg:
        out["learned"] = learned_block(a, w)
    if a.cpu_seconds > 0:
        wc = w.replace(mg_levels=a.mg_levels, mg_steps=a.mg_steps or 5) if mg else w
        out["cpu_baseline"] = cpu_baseline(wc, a.cpu_seconds, wcfg["cpu_stride"], wcfg["cpu_stride_1core"])
    print(json.dumps(out), flush=True)


def learned_block(a, w):
    """Time to 1 % RMS error, learned vs plain, with the allocation network committed for this
    workload (trained by `bench.py --learned <workload>`), on held-out fields 1000, 1001, ..."""
    import numpy as np
    from paper_1810_00188_amd import allocators, inputs, learned, rmc

    try:
        net = allocators.load(a.workload)
    except FileNotFoundError as e:
        return {"error": str(e)}
    gen = {"dns256": inputs.dns256, "channel64": inputs.channel64}[a.workload]
    nu_c, gx = learned.spectral_inputs(w.kd)
    s_plain = rmc.Solver(0)
    s_learn = rmc.Solver(0)
    results = []
    t_start = time.perf_counter()
    for e in range(a.learned_fields):
        we = gen(field_seed=1000 + e)
        s_plain.set_workload(we, device_fields=True)
        s_learn.set_workload(we, device_fields=True, sampling=rmc.SAMPLING_LEARNED, mix_eps=net["mix_eps"])
        s_learn.set_allocator(net["params"], net["mu"], net["sd"], nu_c, gx)
        r = learned.time_to_error(we, s_plain, s_learn, net["mix_eps"], Rs=(16, 32, 64, 128), alloc_cache=1)
        results.append(r)
        row = {"field": 1000 + e}
        for m in ("plain", "learned"):
            row[m] = {k: r[m][k] for k in ("rel_err", "steps_per_ray", "err_slope", "R_target", "t0_s", "t_per_ray_s",
                                           "time_to_target_s", "computes_merged", "t_first_s",
                                           "time_to_target_merged_s")}
        print(f"[learned] field {json.dumps(row)}", file=sys.stderr, flush=True)
    s_plain.close()
    s_learn.close()
    tp = np.array([r["plain"]["time_to_target_merged_s"] for r in results])
    tl = np.array([r["learned"]["time_to_target_merged_s"] for r in results])
    tp1 = np.array([r["plain"]["time_to_target_s"] for r in results])
    tl1 = np.array([r["learned"]["time_to_target_s"] for r in results])
    med = lambda k, m: float(np.median([r[m][k] for r in results]))  # noqa: E731
    return {"metric": "wall time to 1% RMS divq error, as computes of 255 rays per cell: "
                      "ceil(R_1% / 255) (t0 + 255 t1), R_1% and t(R) = t0 + t1 R measured at R = 16..128",
            "unit": "s", "higher_is_better": False,
            "learned_s": float(np.median(tl)), "plain_s": float(np.median(tp)),
            "speedup_vs_plain": float(np.median(tp / tl)), "learned_wins": int(np.sum(tl < tp)),
            "single_compute_model": {"learned_s": float(np.median(tl1)), "plain_s": float(np.median(tp1)),
                                     "speedup_vs_plain": float(np.median(tp1 / tl1)),
                                     "note": "t0 + t1 R_1%, as if one compute carried all R_1% rays per cell"},
            "eval_fields": len(results), "field_seeds": [1000 + e for e in range(len(results))],
            "R_1pct": {"plain": med("R_target", "plain"), "learned": med("R_target", "learned")},
            "t0_s": {"plain": med("t0_s", "plain"), "learned": med("t0_s", "learned")},
            "err_slope": {"plain": med("err_slope", "plain"), "learned": med("err_slope", "learned")},
            "rel_err_R64": {"plain": med_i(results, "plain", 2), "learned": med_i(results, "learned", 2)},
            "reference_rays_per_cell": results[0]["ref_rays_per_cell"],
            "network": net["info"], "eval_s": time.perf_counter() - t_start}


def med_i(results, m, i):
    import numpy as np
    return float(np.median([r[m]["rel_err"][i] for r in results]))


if __name__ == "__main__":
    main()
