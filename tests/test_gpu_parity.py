"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the same seeded
inputs.  FP64 march: per ray within 1e-12 of the oracle; FP32 march: per ray within 1e-5,
both relative to the ray's scale sum tau alpha |I_c - I_j| (+ wall and residual terms);
decisions (band, g-point, octant, ordinal, step counts) identical."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no ROCm GPU visible", allow_module_level=True)

import oracle  # noqa: E402
from paper_1810_00188_amd import inputs, rmc  # noqa: E402

from _parity import (TOL32, TOL64, _check_fp32_rays, _check_fp64_rays, _small_channel,  # noqa: E402
                     _solver, _wall_scale, say)


# ----------------------------------------------------------------------- spectral pdf
def test_plain_pdf_bitwise():
    w = _small_channel()
    say(f"pdf bitwise {w.name}")
    s = _solver(w)
    s.compute()
    p, cb, cg, tm = s.pdf()
    ref = oracle.plain_pdf(oracle.Problem(w))
    assert tm == ref.Tmax
    assert np.array_equal(p, ref.p) and np.array_equal(cb, ref.cdf_b) and np.array_equal(cg, ref.cdf_g)


# -------------------------------------------------------------------------- FP64 parity
@pytest.mark.parametrize("shape", [(10, 7, 6), (5, 9, 3), (1, 4, 1), (13, 2, 17)])
def test_trace_fp64_matches_oracle_per_ray(shape):
    w = _small_channel(nx=shape[0], ny=shape[1], nz=shape[2])
    say(f"trace fp64 {w.name}")
    s = _solver(w)
    cells = np.arange(w.ncells)
    got = s.trace(cells)
    ref = oracle.trace_cells(oracle.Problem(w), cells)
    for f in ("n", "g", "o", "k", "steps", "end"):
        np.testing.assert_array_equal(got[f], ref[f], err_msg=f)
    assert np.array_equal(got["p"], ref["p"])
    _check_fp64_rays(w, cells, got["Y"], ref)


@pytest.mark.parametrize("R", [16, 24, 64])
def test_compute_fp64_matches_oracle(R):
    """Production pipeline (bucketed work list, march kernel, FP64 reduction): every ray slot
    and every cell estimate against the oracle.  The scatter ranks a ray among its cell's equal
    draws by ballots where R divides 64 (16, 64) and from the buckets in LDS otherwise (24); the
    rank keys the ray's direction, so a wrong one shows in the ray values."""
    w = _small_channel(nx=14, ny=11, nz=9, R=R)
    say(f"compute fp64 {w.name}")
    s = _solver(w)
    dq, se = s.compute()
    P = oracle.Problem(w)
    rdq, rse, rsteps = oracle.divergence(P)
    ref = oracle.trace_cells(P, np.arange(w.ncells))
    Y, S = s.ray_values(np.arange(w.ncells))
    np.testing.assert_array_equal(S, ref["steps"])
    _check_fp64_rays(w, np.arange(w.ncells), Y, ref)
    cell_scale = ref["absY"].mean(axis=1) + 1e-300
    assert (np.abs(dq - rdq) / cell_scale).max() < TOL64
    assert (np.abs(se - rse) / cell_scale).max() < 1e-9
    st = s.stats()
    assert st["steps"] == rsteps and st["rays"] == w.ncells * w.R and st["capped_rays"] == 0


@pytest.mark.parametrize("ng", [16, 20])
def test_compute_fp64_large_tables_matches_oracle(ng):
    """100 bands x 16 g (the DNS-size table shape) and x 20 g on a small grid.  With 16 g the
    counting pass stages both cdfs in LDS beside the 12,800 bucket counters (64,816 of 65,536
    bytes); with 20 g (16,000 counters) only the band cdf fits, and a row of the g cdf is ranked
    in global memory.  Ray slots and cell estimates against the oracle."""
    w = _small_channel(nx=6, ny=5, nz=4, R=16, nb=100, ng=ng)
    say(f"compute fp64 {w.name}")
    s = _solver(w)
    dq, se = s.compute()
    P = oracle.Problem(w)
    rdq, rse, rsteps = oracle.divergence(P)
    cells = np.arange(w.ncells)
    ref = oracle.trace_cells(P, cells)
    Y, S = s.ray_values(cells)
    np.testing.assert_array_equal(S, ref["steps"])
    _check_fp64_rays(w, cells, Y, ref)
    cell_scale = ref["absY"].mean(axis=1) + 1e-300
    assert (np.abs(dq - rdq) / cell_scale).max() < TOL64
    assert s.stats()["steps"] == rsteps


def test_grey_slab_full_grid():
    """Grey isothermal slab, 32^3 on 1 x 2 x 1 m, kappa = 1, T = 1000 K, R = 16, FP64."""
    w = inputs.grey_slab(n=32, R=16)
    say(f"grey slab {w.name}")
    s = _solver(w)
    dq, se = s.compute()
    rdq, rse, rsteps = oracle.divergence(oracle.Problem(w))
    assert np.abs(dq - rdq).max() <= TOL64 * 4 * inputs.SIGMA * 1e12
    assert s.stats()["steps"] == rsteps


# -------------------------------------------------------------------------- FP32 parity
def test_trace_fp32_within_1e5():
    w = _small_channel(march="f32", nx=12, ny=10, nz=8, R=16, amp=0.05)
    say(f"trace fp32 {w.name}")
    s = _solver(w)
    cells = np.arange(w.ncells)
    got = s.trace(cells)
    ref = oracle.trace_cells(oracle.Problem(w), cells)
    for f in ("n", "g", "o", "k"):
        np.testing.assert_array_equal(got[f], ref[f], err_msg=f)
    _check_fp32_rays(w, cells, got["Y"], got["steps"], ref)


def test_channel64_sampled_production_launch():
    """Non-grey channel at full size (64^3, 20 bands x 7 g, R = 32, FP32 march, FP64 sums),
    in the launch configuration the benchmark times: every ray slot of all 262,144 cells
    against the oracle's trace (per-ray FP32 bar), and every cell estimate and standard error
    against the oracle's own full run (oracle.divergence) within the mean, respectively the
    propagated, per-ray bar of the cell's rays."""
    w = inputs.channel64()
    say(f"channel64 {w.name}")
    s = _solver(w, device_fields=True)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device="cuda:0")
    se = torch.zeros_like(dq)
    s.compute(dq, se)
    torch.cuda.synchronize()
    P = oracle.Problem(w)
    cells = np.arange(w.ncells)
    ref = oracle.trace_cells(P, cells)
    say(f"channel64 longest ray {ref['steps'].max()} steps")
    Y, S = s.ray_values(cells)
    _check_fp32_rays(w, cells, Y, S, ref)
    # cell estimates: the mean of R rays, each within its per-ray bar b_r, is within mean_r b_r
    # of the oracle's mean; the standard error (a 1-Lipschitz function of the centred ray
    # vector in the l2 norm, over sqrt(R (R - 1))) within ||b||_2 / sqrt(R (R - 1))
    thr = w.tol * _wall_scale(w, ref, cells)
    same = S == ref["steps"]
    b = TOL32 * ref["absY"] + np.where(same, thr * (2.0 ** -52 / w.tol), 2.0 * thr)
    rdq, rse, rsteps = oracle.divergence(P)
    got, got_se = dq.cpu().numpy(), se.cpu().numpy()
    R = w.R
    bar_q = b.mean(axis=1) * (1 + 1e-9) + 1e-300
    bar_se = np.sqrt((b ** 2).sum(axis=1) / (R * (R - 1))) * (1 + 1e-9) + 1e-300
    eq, ese = np.abs(got - rdq), np.abs(got_se - rse)
    rms = np.sqrt(np.mean(rdq ** 2))
    say(f"channel64 cells: max |dq - oracle| / bar {np.max(eq / bar_q):.3f}, / rms(q) {eq.max() / rms:.2e}; "
        f"max |se - oracle| / bar {np.max(ese / bar_se):.3f}")
    assert np.all(eq <= bar_q) and np.all(ese <= bar_se)
    st = s.stats()
    say(f"channel64 stats {st}; oracle steps {rsteps}")
    assert st["rays"] == w.ncells * w.R
    assert abs(st["steps"] - rsteps) <= np.sum(np.abs(S - ref["steps"]))


@pytest.mark.parametrize("after,form", [(1, 0), (4, 0), (37, 0), (1, 1), (37, 1), (1, 2), (37, 2)])
def test_segmented_long_rays_match_oracle(after, form):
    """Rays still marching after `after` steps are finished in parallel segments (form 1: a
    workgroup and 256 segments per ray, 2: a wavefront and 64, 0: by their count): with a tiny
    threshold nearly every ray takes that path; all must match the oracle."""
    w = _small_channel(march="f32", nx=12, ny=10, nz=8, R=16, amp=0.05)
    import dataclasses
    w = w.replace(kd=dataclasses.replace(w.kd, k=w.kd.k * np.float32(0.05)))   # long paths
    say(f"segmented march after {after} steps, form {form}")
    s = _solver(w, long_ray_steps=after, long_ray_form=form)
    s.compute()
    cells = np.arange(w.ncells)
    Y, S = s.ray_values(cells)
    ref = oracle.trace_cells(oracle.Problem(w), cells)
    say(f"oracle steps max {ref['steps'].max()} mean {ref['steps'].mean():.1f}")
    _check_fp32_rays(w, cells, Y, S, ref)


def test_segmented_rounds_with_transparent_slab():
    """A slab with no absorbing gas makes the smallest kappa of the field zero, so only the
    wall, the optical depth seen so far and the step cap bound a round; rays that start in
    or cross the slab need several rounds.  All must match the oracle."""
    w = _small_channel(march="f32", nx=12, ny=10, nz=8, R=16, amp=0.05)
    import dataclasses
    w = w.replace(kd=dataclasses.replace(w.kd, k=w.kd.k * np.float32(0.05)))
    X = np.array(w.X, dtype=np.float64, copy=True).reshape(w.kd.ns, w.nx, w.ny, w.nz)
    X[:, :, 3:6, :] = 0.0
    w = w.replace(X=X.reshape(w.kd.ns, -1))
    say("segmented march, transparent slab, after 2 steps")
    s = _solver(w, long_ray_steps=2)
    s.compute()
    cells = np.arange(w.ncells)
    Y, S = s.ray_values(cells)
    ref = oracle.trace_cells(oracle.Problem(w), cells)
    say(f"oracle steps max {ref['steps'].max()} mean {ref['steps'].mean():.1f}")
    _check_fp32_rays(w, cells, Y, S, ref)


# ----------------------------------------------------------------- properties, edges
def test_rerun_is_bitwise_identical():
    w = _small_channel(march="f32", nx=16, ny=16, nz=16, R=8)
    say(f"determinism {w.name}")
    s = _solver(w)
    a, ae = s.compute()
    b, be = s.compute()
    assert np.array_equal(a, b) and np.array_equal(ae, be)


def test_launch_order_does_not_change_results():
    """The XCD-aware chunk order (and the plain order it reduces to), the sort of each
    bucket's rays by expected length, the regions of the work list (one per snapshot, one per
    brick row, the default) and the allocation tile size only reschedule rays: ray values, step
    counts and cell estimates are bitwise the same."""
    w = _small_channel(march="f32", nx=24, ny=16, nz=20, R=16)
    say(f"xcd spans {w.name}")
    out = []
    for span, lsort, border, tile, region in ((4, 0, 0, 0, -1), (4, 1, 0, 512, 0), (16, 1, 1, 320, 64),
                                              (1024, 0, 1, 65536, 64), (256, 0, 0, 256, 640), (64, 0, 0, 0, 0),
                                              (256, 1, 0, 0, 64)):
        s = _solver(w, xcd_span=span, length_sort=lsort, bucket_order=border, alloc_tile=tile, region_cells=region)
        dq, se = s.compute()
        Y, S = s.ray_values(np.arange(w.ncells))
        out.append((dq, se, Y, S))
    for dq, se, Y, S in out[1:]:
        assert np.array_equal(dq, out[0][0]) and np.array_equal(se, out[0][1])
        assert np.array_equal(Y, out[0][2]) and np.array_equal(S, out[0][3])


@pytest.mark.parametrize("case", ["sparse_runs", "channel64", "channel64_multigrid", "walls", "batch"])
def test_length_sorted_workgroups_keep_results(case):
    """length_sort 1 (each march workgroup sorts the rays of its four chunks by a class of their
    expected length) with regions of the work list only reorders work: cell estimates, ray
    values and step counts are bitwise those of cell order.  sparse_runs: 2 rays per cell in
    one-brick-row regions, so most (region, bucket) runs hold a ray or two and runs of one
    bucket in neighbouring regions meet inside a workgroup's four chunks."""
    say(f"length-sorted runs {case}")
    if case == "batch":
        ws = [_small_channel(march="f32", nx=24 + 8 * q, ny=16 + q, nz=20, R=16, field_seed=q).replace(snap=q)
              for q in range(3)]
        ws = [x.replace(kd=ws[0].kd) for x in ws]
        res = []
        for ls, reg in ((0, -1), (1, 64), (1, 0)):
            solvers = [_solver(x, length_sort=ls, region_cells=reg, long_ray_form=2) for x in ws]
            outs = [np.zeros(x.ncells) for x in ws]
            rmc.compute_batch(solvers, outs)
            res.append(outs)
        for other in res[1:]:
            for a, b in zip(res[0], other):
                assert np.array_equal(a, b)
        return
    kw = {}
    if case == "sparse_runs":
        w = _small_channel(march="f32", nx=20, ny=12, nz=16, R=2)
        variants = ((0, -1), (1, 64), (1, 0))
    elif case == "walls":
        w = _small_channel(march="f32", nx=32, ny=24, nz=28, R=16).replace(eps_walls=(0.5, 0.7))
        variants = ((0, -1), (1, 0), (1, 4096))
    else:
        w = inputs.channel64()
        kw = dict(mg_levels=3) if case == "channel64_multigrid" else {}
        variants = ((0, -1), (1, 0), (1, 65536))
    out = []
    for ls, reg in variants:
        s = _solver(w, length_sort=ls, region_cells=reg, long_ray_form=2, **kw)
        dq, se = s.compute()
        cells = np.arange(0, w.ncells, 7)
        Y, S = s.ray_values(cells)
        out.append((dq, se, Y, S, s.stats()))
    for dq, se, Y, S, st in out[1:]:
        assert np.array_equal(dq, out[0][0]) and np.array_equal(se, out[0][1])
        assert np.array_equal(Y, out[0][2]) and np.array_equal(S, out[0][3])
        assert st["steps"] == out[0][4]["steps"] and st["rays"] == out[0][4]["rays"]


def test_set_fields_equals_separate_ingest():
    """rmc_set_fields (both fields, one synchronisation) gives the compute of
    set_temperature + set_species bitwise, from host arrays and from device tensors; its
    range errors name the field and leave the context usable."""
    import torch
    w = _small_channel(march="f32", nx=12, ny=10, nz=8, R=8)
    say(f"set_fields {w.name}")
    s = _solver(w)
    ref, _ = s.compute()
    T = np.ascontiguousarray(w.T, dtype=np.float32)
    X = np.ascontiguousarray(np.atleast_2d(w.X), dtype=np.float32)
    s.set_temperature(np.full_like(T, 500.0))          # something else in between
    s.set_fields(T, X)
    got, _ = s.compute()
    assert np.array_equal(got, ref)
    dev = torch.device("cuda", 0)
    s.set_fields(torch.from_numpy(T).to(dev), torch.from_numpy(X).to(dev))
    got, _ = s.compute()
    assert np.array_equal(got, ref)
    Tbad = T.copy()
    Tbad[3] = np.nan
    with pytest.raises(rmc.RmcError) as e:
        s.set_fields(Tbad, X)
    assert e.value.status == rmc.RMC_OUT_OF_RANGE and "temperature" in str(e.value)
    Xbad = X.copy()
    Xbad[0, 5] = -1.0
    with pytest.raises(rmc.RmcError) as e:
        s.set_fields(T, Xbad)
    assert e.value.status == rmc.RMC_OUT_OF_RANGE and "mole fractions" in str(e.value)
    s.set_fields(T, X)
    got, _ = s.compute()
    assert np.array_equal(got, ref)


def test_autotune_keeps_results_and_caches(tmp_path):
    """The autotuner only picks schedule knobs: the estimate after tuning is bitwise the
    estimate before; its choice is written to the cache and read back."""
    w = _small_channel(march="f32", nx=20, ny=16, nz=12, R=8)
    say(f"autotune {w.name}")
    s = _solver(w)
    before, _ = s.compute()
    cache = str(tmp_path / "tune.txt")
    got = s.autotune(reps=1, cache_path=cache)
    assert got["xcd_span"] in (16, 64, 256, 1024) and got["length_sort"] in (0, 1)
    assert got["alloc_tile"] in (0, 512)          # 3840 padded cells: automatic tile 256
    after, _ = s.compute()
    assert np.array_equal(before, after)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f": {got['xcd_span']} {got['length_sort']} {got['alloc_tile']}")
    s2 = _solver(w)
    assert s2.autotune(reps=1, cache_path=cache) == got          # a cache hit: no new line
    assert len(open(cache).read().splitlines()) == 1


def test_uniform_temperature_exact_zero():
    w = _small_channel(march="f32")
    w = w.replace(T=np.full(w.ncells, 700.0), T_walls=(700.0, 700.0))
    say("uniform T")
    s = _solver(w)
    dq, se = s.compute()
    assert np.all(dq == 0.0) and np.all(se == 0.0)


def test_device_and_host_fields_agree():
    w = _small_channel(march="f32", R=8)
    say("device vs host fields")
    a, _ = _solver(w).compute()
    s = _solver(w, device_fields=True)
    dq = torch.zeros(w.ncells, dtype=torch.float64, device="cuda:0")
    s.compute(dq)
    torch.cuda.synchronize()
    assert np.array_equal(a, dq.cpu().numpy())


@pytest.mark.parametrize("accum", ["comp32", "f32"])
def test_float_accumulation_modes(accum):
    w = _small_channel(march="f32", R=64)
    say(f"accum {accum}")
    ref, _ = _solver(w).compute()
    got, _ = _solver(w.replace(accum=accum)).compute()
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= (1e-6 if accum == "comp32" else 1e-5) * scale


def test_single_ray_per_cell_and_tiny_grid():
    w = _small_channel(nx=1, ny=1, nz=1, R=1)
    say("1x1x1, R=1")
    s = _solver(w)
    dq, se = s.compute()
    rdq, _, _ = oracle.divergence(oracle.Problem(w))
    assert se[0] == 0.0
    assert abs(dq[0] - rdq[0]) <= TOL64 * abs(rdq[0]) + 1e-300


def test_errors_are_reported_not_fatal():
    w = _small_channel()
    say("error paths")
    s = rmc.Solver(0)
    with pytest.raises(rmc.RmcError) as e:
        s.compute()
    assert e.value.status == rmc.RMC_BAD_STATE
    s.set_grid(w.xf, w.yf, w.zf)
    s.set_walls(*w.T_walls)
    for bad in ((300.0, 300.0, 1.5, 1.0), (300.0, 300.0, 1.0, -0.2)):
        with pytest.raises(rmc.RmcError) as e:
            s.set_walls(*bad)
        assert e.value.status == rmc.RMC_INVALID_ARG
    s.set_kdist(w.kd)
    T = w.T.copy()
    T[5] = 5000.0
    with pytest.raises(rmc.RmcError) as e:
        s.set_temperature(T)
    assert e.value.status == rmc.RMC_OUT_OF_RANGE
    T[5] = np.nan
    with pytest.raises(rmc.RmcError) as e:
        s.set_temperature(T)
    assert e.value.status == rmc.RMC_OUT_OF_RANGE
    X = w.X.copy()
    X[0, 3] = -0.1
    with pytest.raises(rmc.RmcError) as e:
        s.set_species(X)
    assert e.value.status == rmc.RMC_OUT_OF_RANGE
    for bad in (dict(rays_per_cell=0), dict(xcd_span=2), dict(xcd_span=48), dict(long_ray_steps=-1),
                dict(length_sort=2), dict(region_cells=-2), dict(region_cells=32), dict(mg_levels=-2), dict(mg_levels=9), dict(mg_steps=-1),
                dict(alloc_tile=192), dict(alloc_tile=300), dict(alloc_tile=65600), dict(long_ray_form=3)):
        with pytest.raises(rmc.RmcError) as e:
            s.set_options(rmc.default_options(**bad))
        assert e.value.status == rmc.RMC_INVALID_ARG, bad
    # still usable afterwards
    s.set_temperature(w.T)
    s.set_species(w.X)
    s.set_options(rmc.default_options(rays_per_cell=4, march=rmc.F64))
    dq, _ = s.compute()
    assert np.all(np.isfinite(dq))


# ------------------------------------------------------------------ per-cell pdf mode
def test_cell_pdf_mode_matches_oracle():
    w = _small_channel(nx=6, ny=5, nz=4, R=24, nb=3, ng=2)
    rng = np.random.default_rng(9)
    q = rng.gamma(0.5, size=(w.ncells, 3, 2, 8))
    say("cell pdf mode")
    s = _solver(w, sampling=rmc.SAMPLING_PDF, mix_eps=0.2)
    s.set_cell_pdf(q)
    cells = np.arange(w.ncells)
    got = s.trace(cells)
    P = oracle.Problem(w, q_cell=q, mix_eps=0.2)
    ref = oracle.trace_cells(P, cells)
    for f in ("n", "g", "o", "k", "steps", "end"):
        np.testing.assert_array_equal(got[f], ref[f], err_msg=f)
    assert np.array_equal(got["p"], ref["p"])
    _check_fp64_rays(w, cells, got["Y"], ref)
    dq, _ = s.compute()
    rdq, _, _ = oracle.divergence(P)
    assert (np.abs(dq - rdq) / (ref["absY"].mean(axis=1) + 1e-300)).max() < TOL64


# ------------------------------------------------------------------------------ batch
@pytest.mark.parametrize("region", [0, 64])
def test_batch_equals_single_snapshots(region):
    """A batch of three snapshots of different grids equals the single-snapshot computes
    bitwise, with the default regions and with one region per brick row (regions numbered over
    the whole batch)."""
    ws = [_small_channel(march="f32", nx=8 + 4 * q, ny=6 + q, nz=5, R=8, field_seed=q)
          .replace(snap=q) for q in range(3)]
    kd = ws[0].kd
    ws = [x.replace(kd=kd) for x in ws]
    say(f"batch of 3, region_cells {region}")
    singles = [_solver(x).compute()[0] for x in ws]
    solvers = [_solver(x, region_cells=region) for x in ws]
    outs = [np.zeros(x.ncells) for x in ws]
    rmc.compute_batch(solvers, outs)
    for a, b in zip(singles, outs):
        assert np.array_equal(a, b)


def test_batch_of_one_grid_shares_its_face_tables():
    """14 snapshots of one 1000 x 4 x 120 grid: 14 face tables would exceed the LDS a workgroup
    has, one shared table fits; the batch equals the single-snapshot computes bitwise (one
    long-ray form for all: the automatic choice depends on how many long rays a pass has)."""
    ws = [_small_channel(march="f32", nx=1000, ny=4, nz=120, R=2, field_seed=q).replace(snap=q) for q in range(14)]
    kd = ws[0].kd
    ws = [x.replace(kd=kd) for x in ws]
    say("batch of 14 snapshots of one grid")
    singles = [_solver(x, long_ray_form=2).compute()[0] for x in ws]
    solvers = [_solver(x, long_ray_form=2) for x in ws]
    outs = [np.zeros(x.ncells) for x in ws]
    rmc.compute_batch(solvers, outs)
    for a, b in zip(singles, outs):
        assert np.array_equal(a, b)


def test_batch_of_distinct_grids_beyond_64_kib_of_lds():
    """Seven distinct grids whose face tables and table slots need 73 KiB of LDS (more than the
    64 KiB a workgroup had on earlier GPUs; the compute sizes its budget from the device):
    the batch equals the single-snapshot computes bitwise (one long-ray form for all)."""
    ws = [_small_channel(march="f32", nx=1000 - 8 * q, ny=4, nz=120, R=2, field_seed=q).replace(snap=q)
          for q in range(7)]
    kd = ws[0].kd
    ws = [x.replace(kd=kd) for x in ws]
    say("batch of 7 distinct grids, 73 KiB of LDS")
    singles = [_solver(x, long_ray_form=2).compute()[0] for x in ws]
    solvers = [_solver(x, long_ray_form=2) for x in ws]
    outs = [np.zeros(x.ncells) for x in ws]
    rmc.compute_batch(solvers, outs)
    for a, b in zip(singles, outs):
        assert np.array_equal(a, b)


def test_batch_autotune_keeps_results_and_sets_every_context(tmp_path):
    """The batch autotuner times batched passes, writes one cache line naming every grid, and
    sets the chosen schedule on every context; the batched estimate is bitwise unchanged."""
    ws = [_small_channel(march="f32", nx=12 + 4 * q, ny=8, nz=6 + 2 * q, R=8, field_seed=q)
          .replace(snap=q) for q in range(3)]
    kd = ws[0].kd
    ws = [x.replace(kd=kd) for x in ws]
    say("batch autotune of 3")
    solvers = [_solver(x) for x in ws]
    before = [np.zeros(x.ncells) for x in ws]
    rmc.compute_batch(solvers, before)
    cache = str(tmp_path / "tune.txt")
    got = rmc.autotune_batch(solvers, reps=1, cache_path=cache)
    for s in solvers:
        o = s.options()
        assert (o.xcd_span, o.length_sort, o.alloc_tile) == (got["xcd_span"], got["length_sort"], got["alloc_tile"])
    assert [s.options().snapshot for s in solvers] == [0, 1, 2]
    after = [np.zeros(x.ncells) for x in ws]
    rmc.compute_batch(solvers, after)
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and " 12x8x6 16x8x8 20x8x10 : " in lines[0]
    assert rmc.autotune_batch(solvers, reps=1, cache_path=cache) == got
    assert len(open(cache).read().splitlines()) == 1


# ------------------------------------------------------------------------- HIP graphs
@pytest.mark.parametrize("variant", ["plain", "multigrid_reflecting", "closed_box"])
def test_graph_replays_match_eager(variant):
    """Capture one compute of a 2-snapshot batch, replay it several times with eager work and
    synchronisations between the replays, and with new temperature fields set between
    replays; every replay equals an eager compute of the same fields.  Also with the
    multigrid march and reflecting walls (coarse-field kernels and segmented long rays in the
    graph), and in closed boxes."""
    ws = [_small_channel(march="f32", nx=8, ny=6, nz=6, R=8, field_seed=q).replace(snap=q) for q in range(2)]
    kd = ws[0].kd
    ws = [x.replace(kd=kd) for x in ws]
    if variant == "multigrid_reflecting":
        ws = [x.replace(mg_levels=2, mg_steps=2, eps_walls=(0.4, 0.8)) for x in ws]
    elif variant == "closed_box":
        ws = [x.replace(closed=True, T_walls_x=(400.0, 700.0), eps_walls_x=(1.0, 0.5), T_walls_z=(500.0, 800.0),
                        eps_walls_z=(0.3, 1.0)) for x in ws]
    say(f"graph capture and replays ({variant})")
    dev = torch.device("cuda", 0)
    solvers = [_solver(x, device_fields=True) for x in ws]
    outs = [torch.zeros(x.ncells, dtype=torch.float64, device=dev) for x in ws]
    errs = [torch.zeros_like(o) for o in outs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = rmc.Graph(solvers, outs, errs)
    eager_solvers = [_solver(x) for x in ws]
    for rep in range(3):
        if rep > 0:   # new fields for the next replay
            for q, (sv, es) in enumerate(zip(solvers, eager_solvers)):
                T = ws[q].T * (1.0 + 0.01 * rep)
                sv.set_temperature(torch.from_numpy(T.astype(np.float32)).to(dev))
                es.set_temperature(T.astype(np.float32))
        with torch.cuda.stream(stream):
            g.launch()
        stream.synchronize()
        _ = (torch.ones(1000, device=dev) * 2).sum().item()      # eager work between replays
        for q, es in enumerate(eager_solvers):
            ref, ref_se = es.compute()
            assert np.array_equal(outs[q].cpu().numpy(), ref), (rep, q)
            assert np.array_equal(errs[q].cpu().numpy(), ref_se), (rep, q)
    # a changed option invalidates the graph
    solvers[0].set_options(rmc.default_options(rays_per_cell=8, march=rmc.F32, seed=3))
    with pytest.raises(rmc.RmcError) as e:
        g.launch(stream=stream.cuda_stream)
    assert e.value.status == rmc.RMC_BAD_STATE
    g.close()


def test_graph_keeps_its_tables_when_the_leader_works_eagerly():
    """A captured 2-snapshot graph reads its own copies of the planned tables (snapshot
    descriptors, faces, tile map, bucket order, kappa bounds): a trace, a single-snapshot
    compute and a wall-flux compute led by its first context between replays (which rewrite
    that context's tables) leave every replay equal to an eager compute."""
    ws = [_small_channel(march="f32", nx=8 + 4 * q, ny=6, nz=6, R=8, field_seed=q).replace(snap=q) for q in range(2)]
    kd = ws[0].kd
    ws = [x.replace(kd=kd) for x in ws]
    say("graph tables vs eager work of the leader")
    dev = torch.device("cuda", 0)
    solvers = [_solver(x, device_fields=True) for x in ws]
    outs = [torch.zeros(x.ncells, dtype=torch.float64, device=dev) for x in ws]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = rmc.Graph(solvers, outs)
    refs = [_solver(x).compute()[0] for x in ws]
    for rep in range(3):
        if rep == 0:
            solvers[0].trace(np.arange(5))
        elif rep == 1:
            solvers[0].compute()
        else:
            solvers[0].compute_wall_flux()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g.launch()
        stream.synchronize()
        for q in range(2):
            assert np.array_equal(outs[q].cpu().numpy(), refs[q]), (rep, q)
    g.close()


def test_gather_probe_reports_the_access_pattern_rate():
    """The measurement aid of the roofline: needs a previous FP32 compute, then returns the
    kernel time and the bytes of ncells x R lanes x steps gathers (one 16-byte cell record per
    step)."""
    w = _small_channel(march="f32", nx=16, ny=16, nz=16, R=8)
    say("gather probe")
    s = _solver(w)
    with pytest.raises(rmc.RmcError) as e:
        s.gather_probe(10)
    assert e.value.status == rmc.RMC_BAD_STATE
    s.compute()
    ms, by = s.gather_probe(10)
    assert ms > 0.0 and by == w.ncells * w.R * 10 * 16 + (w.ncells * w.R // 64) * 8
    with pytest.raises(rmc.RmcError) as e:
        s.gather_probe(0)
    assert e.value.status == rmc.RMC_INVALID_ARG
