"""Training and evaluation of the learned ray allocation.

This module drives the library; every step of the training (forward pass, loss, backward
pass, Adam) and of the allocation itself (features, network, softmax, draws) runs in its
kernels.  Here are only the choice of data and batches, the schedule, and the measurement of
the wall time the learned and the plain allocation need to reach a given RMS error.

Training data: rays of plain runs (the T_max pdf) on training fields, taken with the
production trace path: per ray its stratum s = (n*ng + g)*8 + o, its probability p0 and
h = Y p0.  The loss (see rmc_train_grad) is the relative second moment of each cell's
estimator under the proposed pdf.

Error of a run: e(R) = sqrt(max(mean_c (q_c - qref_c)^2 - mean_c se_ref,c^2, 0)) / rms(qref),
the RMS deviation from a high-R plain reference with the reference's own variance removed,
relative to the RMS of the reference field.  With e proportional to R^-1/2, the rays per cell
for a 1 % error are R_1 = R (e(R) / 0.01)^2; the wall time per compute is fitted as
t(R) = t0 + t1 R over the measured R, and the time to 1 % is t(R_1).
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import rmc

SHAPES = [(64, 5), (64,), (64, 64), (64,), (64, 64), (64,), (8, 64), (8,)]


def init_params(seed: int, out_scale: float = 0.1) -> np.ndarray:
    """He-uniform weights, zero biases, the output layer scaled by out_scale (float32, in the
    order of rmc_set_allocator)."""
    rng = np.random.default_rng(seed)
    parts = []
    for q, shp in enumerate(SHAPES):
        if len(shp) == 2:
            lim = np.sqrt(6.0 / shp[1])
            w = rng.uniform(-lim, lim, shp)
            if q == 6:
                w = w * out_scale
        else:
            w = np.zeros(shp)
        parts.append(w.ravel())
    return np.concatenate(parts).astype(np.float32)


def spectral_inputs(kd):
    """Band centres (cm^-1) and g abscissae of a table set."""
    return kd.nu_lo + 0.5 * kd.dnu, np.asarray(kd.gx, dtype=np.float64)


def standardisation(feats: Sequence[np.ndarray], kd):
    """(mu, sd) of the five raw inputs over the training cells and the (n, g) pairs."""
    f = np.concatenate(feats).astype(np.float64)
    nu_c, gx = spectral_inputs(kd)
    spec = np.stack(np.broadcast_arrays((nu_c / 1e4)[:, None], gx[None, :]), axis=-1).reshape(-1, 2)
    mu = np.concatenate([f.mean(0), spec.mean(0)])
    sd = np.concatenate([f.std(0), spec.std(0)]) + 1e-3
    return mu.astype(np.float32), sd.astype(np.float32)


@dataclass
class RunSamples:
    """Training rays of one plain run, on the device (torch tensors), R per cell in cell order."""
    feat: object
    mask: object
    pplain: object
    strata: object
    h: object
    p0: object
    ncell: int
    R: int
    cost: object = None         # device: cost of every ray (steps + a fixed overhead)


def plain_samples(s: rmc.Solver, cells: np.ndarray, overhead: float = 5.0) -> RunSamples:
    """Rays of the listed cells under the solver's current fields and plain sampling; the cost
    of a ray is its number of steps plus `overhead` (allocation, set-up and reduction of a
    ray, in step equivalents)."""
    import torch
    dev = torch.device("cuda", s.device)
    rec = s.trace(cells)
    kd_ng = s.ng
    strata = ((rec["n"] * kd_ng + rec["g"]) * 8 + rec["o"]).astype(np.int32).ravel()
    p0 = rec["p"].ravel()
    h = rec["Y"].ravel() * p0
    feat, mask = s.features()
    p, _, _, _ = s.pdf()
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    return RunSamples(T(feat[cells], torch.float32), T(mask[cells], torch.uint8), T(p.ravel(), torch.float64),
                      T(strata, torch.int32), T(h, torch.float64), T(p0, torch.float64), len(cells), s.R,
                      T(rec["steps"].ravel().astype(np.float64) + overhead, torch.float64))


def batch_of(run: RunSamples, sel: np.ndarray, use_cost: bool = True):
    """TrainBatch of the selected cells (indices into the run, sorted) and its keep-alive list."""
    import torch
    dev = run.feat.device
    sel_t = torch.from_numpy(np.ascontiguousarray(sel, dtype=np.int64)).to(dev)
    ridx = (sel_t[:, None] * run.R + torch.arange(run.R, device=dev)[None, :]).reshape(-1)
    cell_of = torch.arange(len(sel), device=dev, dtype=torch.int32).repeat_interleave(run.R)
    return rmc.train_batch(run.feat[sel_t].contiguous(), run.mask[sel_t].contiguous(), run.pplain,
                           cell_of.contiguous(), run.strata[ridx].contiguous(), run.h[ridx].contiguous(),
                           run.p0[ridx].contiguous(),
                           ray_cost=run.cost[ridx].contiguous() if use_cost else None)


def shuffle_run(run: RunSamples, rng) -> list:
    """Reorder a run's cells (with their rays) by a random permutation, in place; returns the
    tensors it held before (kept alive by the caller while queued work may still read them)."""
    import torch
    dev = run.feat.device
    perm = torch.from_numpy(rng.permutation(run.ncell)).to(dev)
    ridx = (perm[:, None] * run.R + torch.arange(run.R, device=dev)[None, :]).reshape(-1)
    old = [run.feat, run.mask, run.strata, run.h, run.p0, run.cost]
    run.feat, run.mask = run.feat[perm].contiguous(), run.mask[perm].contiguous()
    run.strata, run.h, run.p0 = run.strata[ridx].contiguous(), run.h[ridx].contiguous(), run.p0[ridx].contiguous()
    if run.cost is not None:
        run.cost = run.cost[ridx].contiguous()
    return old


def train(s: rmc.Solver, runs: List[RunSamples], steps: int, lr: float, batch_cells: int, seed: int = 0,
          log: Optional[Callable[[str], None]] = None, lr_final: Optional[float] = None,
          use_cost: bool = True, chunk: int = 256) -> List[float]:
    """Adam steps on batches of batch_cells cells taken from the runs in turn; each run's cells
    are visited in a random order, reshuffled at every pass over the run (a batch is then a
    contiguous slice of the run: no per-step gathers).  The learning rate decays geometrically
    to lr_final (default lr / 10).  With use_cost the loss is the work-normalised second
    moment (the rays' costs weigh in).  The steps go to the library `chunk` at a time
    (rmc_train_steps: no synchronisation between them).  Returns the batch losses."""
    import torch
    rng = np.random.default_rng(seed)
    lr_final = lr / 10.0 if lr_final is None else lr_final
    B = {id(r): min(batch_cells, r.ncell) for r in runs}
    pos = {id(r): None for r in runs}
    cell_of = {}
    losses: List[float] = []
    t = 0
    while t < steps:
        n = min(chunk, steps - t)
        batches, keep, lrs = [], [], []
        for q in range(t, t + n):
            run = runs[q % len(runs)]
            b = B[id(run)]
            if pos[id(run)] is None or pos[id(run)] + b > run.ncell:
                keep.append(shuffle_run(run, rng))
                pos[id(run)] = 0
            a0 = pos[id(run)]
            pos[id(run)] = a0 + b
            key = (b, run.R)
            if key not in cell_of:
                cell_of[key] = torch.arange(b, device=run.feat.device, dtype=torch.int32).repeat_interleave(run.R)
            r0, r1 = a0 * run.R, (a0 + b) * run.R
            bt, kp = rmc.train_batch(run.feat[a0:a0 + b], run.mask[a0:a0 + b], run.pplain, cell_of[key],
                                     run.strata[r0:r1], run.h[r0:r1], run.p0[r0:r1],
                                     ray_cost=run.cost[r0:r1] if use_cost else None)
            batches.append(bt)
            keep.append(kp)
            lrs.append(lr * (lr_final / lr) ** (q / max(steps - 1, 1)))
        losses.extend(s.train_steps(batches, lrs).tolist())
        t += n
        if log and (t // chunk) % max(steps // chunk // 10, 1) == 0 or (log and t == steps):
            m = max(min(steps // 10, len(losses)), 1)
            log(f"train step {t}: loss {np.mean(losses[-m:]):.4f} lr {lrs[-1]:.2e}")
    return losses


def rel_error(dq: np.ndarray, qref: np.ndarray, se_ref: np.ndarray) -> float:
    """RMS deviation from the reference with the reference variance removed, relative to the
    RMS of the reference."""
    e2 = np.mean((dq - qref) ** 2) - np.mean(se_ref ** 2)
    return float(np.sqrt(max(e2, 0.0)) / np.sqrt(np.mean(qref ** 2)))


def timed_compute(s: rmc.Solver, dq, reps: int) -> float:
    """Wall time of one compute (mean over reps, device outputs, after one warm-up)."""
    import torch
    s.compute(dq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.compute(dq)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def time_to_error(w, s_plain: rmc.Solver, s_learn: rmc.Solver, mix_eps: float, Rs=(16, 32, 64, 128),
                  ref_runs: int = 8, ref_R: int = 255, reps: int = 2, target: float = 0.01,
                  snap_base: int = 1000, log: Optional[Callable[[str], None]] = None, r_max: int = 255,
                  alloc_cache: int = 0) -> dict:
    """Reference, errors and times at several R for both allocations on one field; the time
    each needs for a `target` relative RMS error: t(R_1%) = t0 + t1 R_1% as if one compute
    carried all R_1% rays per cell, and, as they are run, K = ceil(R_1% / r_max) computes of
    r_max rays each: K (t0 + t1 r_max) (every compute pays t0, the allocation network's cost in
    the learned mode).  With alloc_cache the learned computes reuse the field's allocation pair
    sums (rmc_options.alloc_cache): the network's full pass is paid once per field (t_first, the
    excess of the first compute over a cached one, added to the merged time) and t0 is the
    cached computes' overhead.  s_plain / s_learn carry the field, the tables and their options
    (plain and learned sampling); their R and snapshot are changed here."""
    import torch
    dev = torch.device("cuda", s_plain.device)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device=dev)
    se = torch.zeros_like(dq)

    def set_opts(s, R, snap, sampling, eps):
        s.set_options(rmc.default_options(rays_per_cell=R, seed=w.seed, snapshot=snap, tol=w.tol,
                                          max_steps=w.max_steps, march=rmc.F32, accum=rmc.ACC[w.accum],
                                          sampling=sampling, mix_eps=eps,
                                          alloc_cache=alloc_cache if sampling == rmc.SAMPLING_LEARNED else 0))

    # reference: ref_runs independent plain runs of ref_R rays (distinct snapshot streams)
    qsum = np.zeros(w.ncells)
    v = np.zeros(w.ncells)
    for k in range(ref_runs):
        set_opts(s_plain, ref_R, snap_base + k, rmc.SAMPLING_PLAIN, 0.0)
        s_plain.compute(dq, se)
        torch.cuda.synchronize()
        qsum += dq.cpu().numpy()
        v += se.cpu().numpy() ** 2
    qref = qsum / ref_runs
    se_ref = np.sqrt(v) / ref_runs
    out = {"ref_rays_per_cell": ref_runs * ref_R}
    for name, s, sampling in (("plain", s_plain, rmc.SAMPLING_PLAIN), ("learned", s_learn, rmc.SAMPLING_LEARNED)):
        eps = mix_eps if sampling == rmc.SAMPLING_LEARNED else 0.0
        es, ts, spr = [], [], []
        t_first = 0.0
        if alloc_cache and sampling == rmc.SAMPLING_LEARNED:
            # the first compute of the field fills the cache: its excess over a cached compute
            set_opts(s, Rs[0], snap_base + 99, sampling, eps)
            torch.cuda.synchronize()
            t0_ = time.perf_counter()
            s.compute(dq)
            torch.cuda.synchronize()
            t_first = time.perf_counter() - t0_
            t_first -= timed_compute(s, dq, reps)
        for R in Rs:
            set_opts(s, R, snap_base + 100 + R, sampling, eps)
            ts.append(timed_compute(s, dq, reps))
            es.append(rel_error(dq.cpu().numpy(), qref, se_ref))
            st = s.stats()
            spr.append(st["steps"] / max(st["rays"], 1))
        Rs_a, es_a, ts_a = np.array(Rs, dtype=float), np.array(es), np.array(ts)
        slope = float(np.polyfit(np.log(Rs_a), np.log(np.maximum(es_a, 1e-300)), 1)[0])
        R1 = float(np.median(Rs_a * (es_a / target) ** 2))
        t1, t0 = np.polyfit(Rs_a, ts_a, 1)
        K = max(1, int(np.ceil(R1 / r_max)))
        out[name] = {"R": list(Rs), "rel_err": es, "t_s": ts, "steps_per_ray": spr, "err_slope": slope, "R_target": R1,
                     "t0_s": float(t0), "t_per_ray_s": float(t1), "time_to_target_s": float(t0 + t1 * R1),
                     "computes_merged": K, "t_first_s": float(t_first),
                     "time_to_target_merged_s": float(t_first + K * (t0 + t1 * r_max))}
        if log:
            log(f"{name}: err {np.round(es_a, 5).tolist()} slope {slope:.2f} R_1% {R1:.0f} steps/ray {spr[-1]:.1f} "
                f"t(R) {np.round(ts_a * 1e3, 2).tolist()} ms -> {out[name]['time_to_target_s']:.3f} s "
                f"({K} computes of {r_max}: {out[name]['time_to_target_merged_s']:.3f} s)")
    return out
