"""GPU parity of the learned ray allocation against the FP64 references in oracle/ (the
network, its loss and gradient in oracle.mlp; the draws and ray values in the C oracle's
per-cell-pdf mode).

* Features: float32 storage of an FP64 computation, within 1e-6; gradient masks exact.
* Logits: the hidden layers run on BF16 matrix cores (inputs and weights rounded to BF16,
  unit roundoff u = 2^-8, FP32 accumulation); the test propagates the first-order bound
  e_l = |W_l| e_{l-1} + 2u |W_l| (|h_{l-1}| + e_{l-1}) from the FP64 forward pass and
  requires |z_gpu - z| <= 1.5 e_4 + 1e-5.
* Draws: the oracle receives the kernel's own logits as its per-cell pdf, so only the
  softmax / cumulative sums differ (FP32 exponentials on the device): decisions identical
  for all but a vanishing fraction of rays, probabilities within 1e-5, ray values (FP64
  march) within 1e-6 of their scale.
* Training: loss and gradient of the FP32 kernels against the FP64 chain rule, relative
  error of the gradient vector below 1e-4.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no ROCm GPU visible", allow_module_level=True)

import oracle  # noqa: E402
from oracle import mlp  # noqa: E402
from paper_1810_00188_amd import inputs, rmc  # noqa: E402
from _parity import _wall_scale, say  # noqa: E402

U_BF16 = 2.0 ** -8


def _workload(march="f64", **kw):
    base = dict(nx=10, ny=8, nz=6, R=16, nb=5, ng=3, amp=0.1, stretch=2.0, species_amp=0.2,
                co2=True, march=march)
    base.update(kw)
    return inputs.channel(**base).replace(T_walls=(350.0, 900.0))


def _network(w, feat, seed=3, out_scale=10.0):
    """Seeded parameters (larger output layer so that the pdf is far from uniform) and the
    standardisation of the workload's features."""
    p = mlp.init_params(seed)
    p["W4"] = p["W4"] * out_scale
    p["b4"] = np.linspace(-1.0, 1.0, 8)
    params = mlp.flatten(p).astype(np.float32)
    kd = w.kd
    fs = mlp.spectral_features(kd).reshape(-1, 2)
    allf = np.concatenate([feat.astype(np.float64), np.zeros((len(feat), 2))], axis=1)
    mu = np.concatenate([allf[:, :3].mean(0), fs.mean(0)])
    sd = np.concatenate([allf[:, :3].std(0), fs.std(0)]) + 1e-3
    nu_c = kd.nu_lo + 0.5 * kd.dnu
    return params, mu.astype(np.float32), sd.astype(np.float32), nu_c, kd.gx


def _solver(w, **kw):
    s = rmc.Solver(0)
    s.set_workload(w, **kw)
    return s


def _oracle_logits(w, params, mu, sd, feat, mask):
    p = mlp.unflatten(params.astype(np.float64))
    x = mlp.assemble_inputs(feat.astype(np.float64), mlp.spectral_features(w.kd), mu.astype(np.float64),
                            sd.astype(np.float64))
    z, cache = mlp.forward(p, x)
    return p, x, z, cache


def test_features_match_oracle():
    w = _workload()
    say(f"features {w.name}")
    s = _solver(w)
    feat, mask = s.features()
    f, m = mlp.cell_features(w)
    np.testing.assert_allclose(feat, f.astype(np.float32), rtol=1e-6, atol=1e-6)
    assert np.array_equal(mask, m.astype(np.uint8))


@pytest.mark.parametrize("tables", [(5, 3), (100, 16)])
def test_logits_within_bf16_bound(tables):
    w = _workload(nb=tables[0], ng=tables[1])
    say(f"logits {w.name}")
    s = _solver(w)
    feat, mask = s.features()
    params, mu, sd, nu_c, gx = _network(w, feat)
    s.set_allocator(params, mu, sd, nu_c, gx)
    cells = np.arange(w.ncells)
    zg = s.allocator_logits(cells)
    p, x, z, (x_, a1, h1, a2, h2, a3, h3) = _oracle_logits(w, params, mu, sd, feat, mask)
    ref = mlp.octant_logits(z, mask)
    # first-order propagation of the BF16 roundings through the layers (ReLU is 1-Lipschitz)
    A = {k: np.abs(v) for k, v in p.items()}
    # layer 1 runs in FP32 from FP32 features (standardisation may cancel): a loose floor
    e1 = 1e-5 * ((np.abs(x) + 1.0) @ A["W1"].T + A["b1"])
    e2 = (e1 @ A["W2"].T) + 2 * U_BF16 * ((np.abs(h1) + e1) @ A["W2"].T)
    e3 = (e2 @ A["W3"].T) + 2 * U_BF16 * ((np.abs(h2) + e2) @ A["W3"].T)
    e4 = (e3 @ A["W4"].T) + 2 * U_BF16 * ((np.abs(h3) + e3) @ A["W4"].T)
    bound = mlp.octant_logits(1.5 * e4 + 1e-5, mask)
    err = np.abs(zg.astype(np.float64) - ref)
    say(f"logits: max |dz| {err.max():.3e}, max bound {bound.max():.3e}, max |z| {np.abs(ref).max():.2f}")
    assert np.all(err <= bound)


def _plain_cdf_inverse_check(P, u0, u1, u2, nb, ng):
    """Reference draw of the mixture pdf P[nb*ng*8] (FP64, sequential cumulative sums)."""
    pc = P.reshape(nb, ng, 8)
    tot = pc.sum()
    bn = pc.sum(axis=(1, 2))
    cb = np.cumsum(bn) / tot
    cb[-1] = 1.0
    n = int(np.searchsorted(cb, u0, side="right"))
    gn = pc[n].sum(axis=1)
    cg = np.cumsum(gn) / bn[n]
    cg[-1] = 1.0
    g = int(np.searchsorted(cg, u1, side="right"))
    co = np.cumsum(pc[n, g]) / gn[g]
    co[-1] = 1.0
    o = int(np.searchsorted(co, u2, side="right"))
    return (n * ng + g) * 8 + o, min(np.abs(cb - u0).min(), np.abs(cg - u1).min(), np.abs(co - u2).min())


@pytest.mark.parametrize("tables", [(5, 3), (20, 7), (100, 16)])
def test_learned_draws_and_rays_match_oracle(tables):
    """Draws and ray values of the learned mode.  The table sets cover the kernel's cases: 5 x 3
    (one 16-row network tile per cell), 20 x 7 (9 tiles), and 100 x 16, the DNS-size tables
    (100 tiles and 12,800 strata per cell, band sums and running sums over two 64-band
    chunks)."""
    eps = 0.15
    w = _workload(R=24, nb=tables[0], ng=tables[1])
    say(f"learned sampling {w.name}")
    s = _solver(w)
    feat, mask = s.features()
    params, mu, sd, nu_c, gx = _network(w, feat)
    s = _solver(w, sampling=rmc.SAMPLING_LEARNED, mix_eps=eps)
    s.set_allocator(params, mu, sd, nu_c, gx)
    s.compute()
    cells = np.arange(w.ncells)
    strat, prob = s.ray_draws(cells)
    Y, S = s.ray_values(cells)
    zg = s.allocator_logits(cells).astype(np.float64)
    zp = mlp.prior_logits(zg, oracle.plain_pdf(oracle.Problem(w)).p)     # softmax arguments
    q = np.exp(zp - zp.reshape(len(cells), -1).max(axis=1)[:, None, None, None])
    q /= q.reshape(len(cells), -1).sum(axis=1)[:, None, None, None]
    P = oracle.Problem(w, q_cell=q, mix_eps=eps)
    ref = oracle.trace_cells(P, cells)
    rs = (ref["n"] * w.kd.ng + ref["g"]) * 8 + ref["o"]
    same = strat == rs
    say(f"draws: {np.sum(~same)} of {same.size} differ")
    # every differing draw sits within rounding of a cumulative-sum boundary
    pp = oracle.plain_pdf(P).p
    key = (w.seed & 0xFFFFFFFF, w.seed >> 32)
    for a, r in np.argwhere(~same):
        wd = oracle.philox(np.array([a, r, 0, (w.snap << 4) | 1], dtype=np.uint32), key)
        u = (wd[:3].astype(np.float64) + 0.5) * 2.0 ** -32
        Pm = (1 - eps) * q[a].ravel() + eps * np.repeat(pp.ravel(), 8) / 8
        _, gap = _plain_cdf_inverse_check(Pm, u[0], u[1], u[2], w.kd.nb, w.kd.ng)
        assert gap < 1e-6, (a, r, gap)
    assert np.mean(~same) < 1e-3
    cell_ok = same.all(axis=1)
    np.testing.assert_allclose(prob[same], ref["p"][same], rtol=1e-5)
    # ray values: within 1e-6 of their scale (the FP32 exponentials of the softmax) plus the
    # FP64 rounding floor of the march (alpha one ulp apart where 1 - alpha is a few ulps)
    floor = 2.0 ** -52 * _wall_scale(w, ref, cells)
    d = np.abs(Y - ref["Y"])[cell_ok]
    say(f"ray values: max |dY| / scale {np.max(d / np.maximum(ref['absY'][cell_ok], 1e-300)):.2e}")
    assert np.all(d <= 1e-6 * ref["absY"][cell_ok] + floor[cell_ok] + 1e-300)
    assert np.array_equal(S[cell_ok], ref["steps"][cell_ok])
    # the trace path reads the same draws
    tr = s.trace(cells[:20])
    assert np.array_equal((tr["n"] * w.kd.ng + tr["g"]) * 8 + tr["o"], strat[:20])


def test_allocation_cache_gives_the_same_draws():
    """alloc_cache: the compute that fills the cache and later ones that read it (another
    snapshot, another R) draw exactly what computes without it draw; a new temperature field
    rebuilds it; a captured graph refuses it."""
    eps = 0.15
    w = _workload(R=24, nb=20, ng=7, march="f32")
    say(f"allocation cache {w.name}")
    feat, _ = _solver(w).features()
    params, mu, sd, nu_c, gx = _network(w, feat)
    cells = np.arange(w.ncells)

    def solver(cache):
        s = _solver(w, sampling=rmc.SAMPLING_LEARNED, mix_eps=eps, alloc_cache=cache)
        s.set_allocator(params, mu, sd, nu_c, gx)
        return s

    s_c, s_n = solver(1), solver(0)

    def same(snap, R):
        out = []
        for s, cache in ((s_c, 1), (s_n, 0)):
            s.set_options(rmc.default_options(rays_per_cell=R, seed=w.seed, snapshot=snap, tol=w.tol,
                                              max_steps=w.max_steps, march=rmc.F32, sampling=rmc.SAMPLING_LEARNED,
                                              mix_eps=eps, alloc_cache=cache))
            dq, se = s.compute()
            out.append((s.ray_draws(cells), dq))
        (a_draw, a_q), (b_draw, b_q) = out
        assert np.array_equal(a_draw[0], b_draw[0]) and np.array_equal(a_draw[1], b_draw[1]), (snap, R)
        assert np.array_equal(a_q, b_q), (snap, R)

    same(0, 24)      # fills the cache
    same(5, 16)      # reads it
    same(9, 40)
    T2 = (np.asarray(w.T, dtype=np.float64) * 1.02).astype(np.float32)
    for s in (s_c, s_n):
        s.set_temperature(T2)
    same(11, 24)     # the field changed: rebuilt
    same(12, 24)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with pytest.raises(rmc.RmcError) as e:
            rmc.Graph([s_c], [torch.zeros(w.ncells, dtype=torch.float64, device="cuda:0")])
    assert e.value.status == rmc.RMC_UNSUPPORTED


def test_learned_compute_with_length_sorted_workgroups_keeps_results():
    """Learned sampling (per-ray probabilities) with each march workgroup's rays sorted by
    expected length (length_sort 1) and one-brick-row regions: cell estimates bitwise those of
    cell order."""
    eps = 0.15
    w = _workload(R=24, nb=20, ng=7, march="f32")
    say(f"learned length-sorted runs {w.name}")
    feat, _ = _solver(w).features()
    params, mu, sd, nu_c, gx = _network(w, feat)
    out = []
    for ls in (0, 1):
        s = _solver(w, sampling=rmc.SAMPLING_LEARNED, mix_eps=eps, length_sort=ls, region_cells=64 if ls else -1)
        s.set_allocator(params, mu, sd, nu_c, gx)
        out.append(s.compute())
    for dq, se in out[1:]:
        assert np.array_equal(out[0][0], dq) and np.array_equal(out[0][1], se)


def _training_batch(w, s, ncell, seed=4):
    """Plain-run rays of ncell sampled cells (oracle trace): device tensors of a TrainBatch and
    the host arrays the FP64 reference needs."""
    rng = np.random.default_rng(seed)
    cells = np.sort(rng.choice(w.ncells, ncell, replace=False))
    P = oracle.Problem(w)
    ref = oracle.trace_cells(P, cells)
    strata = ((ref["n"] * w.kd.ng + ref["g"]) * 8 + ref["o"]).ravel().astype(np.int32)
    p0 = ref["p"].ravel()
    h = ref["Y"].ravel() * p0
    cell_of = np.repeat(np.arange(ncell), w.R).astype(np.int32)
    feat, mask = s.features()
    pplain = oracle.plain_pdf(P).p.ravel()
    dev = torch.device("cuda", 0)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)  # noqa: E731
    tens = (T(feat[cells], torch.float32), T(mask[cells], torch.uint8), T(pplain, torch.float64),
            T(cell_of, torch.int32), T(strata, torch.int32), T(h, torch.float64), T(p0, torch.float64))
    return tens, dict(cells=cells, feat=feat[cells], mask=mask[cells], pplain=pplain, cell_of=cell_of,
                      strata=strata, h=h, p0=p0)


@pytest.mark.parametrize("with_cost", [False, True])
def test_training_gradient_matches_oracle(with_cost):
    eps = 0.1
    w = _workload(R=16)
    say(f"training gradient {w.name}")
    s = _solver(w, sampling=rmc.SAMPLING_PLAIN, mix_eps=eps)
    feat, _ = s.features()
    params, mu, sd, nu_c, gx = _network(w, feat, out_scale=3.0)
    s.set_allocator(params, mu, sd, nu_c, gx)
    tens, H = _training_batch(w, s, ncell=40)
    kd = w.kd
    cost = np.random.default_rng(2).uniform(2.0, 40.0, len(H["h"])) if with_cost else None
    ct = torch.from_numpy(cost).to("cuda:0") if with_cost else None
    batch, keep = rmc.train_batch(*tens, ray_cost=ct)
    loss_g, grad_g = s.train_grad(batch)
    p, x, z, cache = _oracle_logits(w, params, mu, sd, H["feat"], H["mask"])
    zg = mlp.octant_logits(z, H["mask"])
    L, dzg = mlp.allocation_loss(zg, H["pplain"].reshape(kd.nb, kd.ng), eps, H["cell_of"], H["strata"], H["h"],
                                 H["p0"], ray_cost=cost)
    dz = mlp.octant_logits(dzg, H["mask"])
    g = mlp.flatten(mlp.backward(p, cache, dz))
    rel = np.linalg.norm(grad_g - g) / np.linalg.norm(g)
    say(f"training: loss gpu {loss_g:.8f} oracle {L:.8f}; gradient rel err {rel:.2e}")
    assert abs(loss_g - L) <= 1e-5 * abs(L)
    assert rel < 1e-4
    # unsorted samples are rejected
    bad = list(tens)
    bad[3] = tens[3].flip(0).contiguous()
    b2, k2 = rmc.train_batch(*bad)
    with pytest.raises(rmc.RmcError) as e:
        s.train_grad(b2)
    assert e.value.status == rmc.RMC_INVALID_ARG


def test_adam_steps_match_oracle():
    """Two rmc_train_step calls from a freshly set allocator (zero Adam moments) against
    oracle.mlp.adam_step (Kingma & Ba) fed the gradient rmc_train_grad returns at the same
    parameters (the training kernels are deterministic, so it is the gradient the step uses).
    Step 1 checks the bias-corrected update from zero moments, step 2 the moment recursions
    (the reference carries its own FP64 moments).  Bar per parameter: FP32 rounding of the
    update and of the stored parameter, 2^-23 |v| + 1e-5 lr (1 + |update| / lr)."""
    eps = 0.1
    lr = float(np.float32(2e-3))
    w = _workload(R=16)
    say(f"adam steps {w.name}")
    s = _solver(w, sampling=rmc.SAMPLING_PLAIN, mix_eps=eps)
    feat, _ = s.features()
    params, mu, sd, nu_c, gx = _network(w, feat, out_scale=3.0)
    s.set_allocator(params, mu, sd, nu_c, gx)
    tens, H = _training_batch(w, s, ncell=40)
    cost = torch.from_numpy(np.random.default_rng(6).uniform(2.0, 40.0, len(H["h"]))).to("cuda:0")
    batch, keep = rmc.train_batch(*tens, ray_cost=cost)
    m = np.zeros(rmc.MLP_PARAMS)
    q = np.zeros(rmc.MLP_PARAMS)
    for t in (1, 2):
        cur = s.get_allocator().astype(np.float64)
        loss_g, g = s.train_grad(batch)
        loss_s = s.train_step(batch, lr)
        got = s.get_allocator().astype(np.float64)
        ref, m, q = mlp.adam_step(cur, g.astype(np.float64), m, q, t, lr=lr)
        upd = np.abs(ref - cur)
        bar = 2.0 ** -23 * np.abs(ref) + 1e-5 * (lr + upd)
        err = np.abs(got - ref)
        say(f"adam step {t}: loss {loss_s:.6f}, max |update| / lr {upd.max() / lr:.3f}, "
            f"max err / bar {np.max(err / bar):.3f}")
        assert loss_s == loss_g
        assert np.all(err <= bar)
        assert np.count_nonzero(upd) > rmc.MLP_PARAMS // 2


def test_training_lowers_the_loss():
    eps = 0.1
    w = _workload(R=16)
    say(f"training steps {w.name}")
    s = _solver(w, sampling=rmc.SAMPLING_PLAIN, mix_eps=eps)
    feat, _ = s.features()
    params, mu, sd, nu_c, gx = _network(w, feat, out_scale=1.0)
    s.set_allocator(params, mu, sd, nu_c, gx)
    tens, _ = _training_batch(w, s, ncell=120, seed=8)
    batch, keep = rmc.train_batch(*tens)
    first = s.train_step(batch, 3e-3)
    for _ in range(150):
        last = s.train_step(batch, 3e-3)
    say(f"training: loss {first:.4f} -> {last:.4f}")
    assert last < 0.9 * first
    assert np.all(np.isfinite(s.get_allocator()))


def test_trained_network_gains_over_plain_on_held_out_field():
    """What the trained network gains: trained by the library's kernels on two fields, on a
    held-out field it reaches a given RMS error of the heat source with less work (error^2 x
    steps per ray at equal R) than the plain allocation, and its error keeps falling as
    R^-1/2 (the importance weights keep it unbiased: no error floor)."""
    from paper_1810_00188_amd import learned
    eps = 0.1

    def gen(fs):
        return inputs.channel(nx=16, ny=16, nz=16, R=32, nb=5, ng=3, amp=0.1, field_seed=fs)

    w0 = gen(1)
    say(f"learned gain {w0.name}")
    s = _solver(w0, mix_eps=eps)
    runs, feats = [], []
    for k, fs in enumerate((1, 2)):
        w = gen(fs)
        s.set_temperature(np.ascontiguousarray(w.T, dtype=np.float32))
        s.set_species(np.ascontiguousarray(w.X, dtype=np.float32))
        s.set_options(rmc.default_options(rays_per_cell=64, seed=w.seed, snapshot=k + 1, tol=w.tol,
                                          max_steps=w.max_steps, march=rmc.F32, mix_eps=eps))
        runs.append(learned.plain_samples(s, np.arange(w.ncells)))
        feats.append(runs[-1].feat.cpu().numpy())
    nu_c, gx = learned.spectral_inputs(w0.kd)
    mu, sd = learned.standardisation(feats, w0.kd)
    s.set_allocator(learned.init_params(0), mu, sd, nu_c, gx)
    losses = learned.train(s, runs, 600, 2e-3, 64)
    params = s.get_allocator()
    s.close()
    w = gen(1000)
    s_plain = _solver(w)
    s_learn = _solver(w, sampling=rmc.SAMPLING_LEARNED, mix_eps=eps)
    s_learn.set_allocator(params, mu, sd, nu_c, gx)
    out = learned.time_to_error(w, s_plain, s_learn, eps, Rs=(16, 64), ref_runs=8, ref_R=255, reps=1)
    pl, le = out["plain"], out["learned"]
    work = [(x["rel_err"][1] ** 2) * x["steps_per_ray"][1] for x in (pl, le)]
    say(f"training loss {np.mean(losses[:20]):.3f} -> {np.mean(losses[-20:]):.3f}; error at R = 64: plain "
        f"{pl['rel_err'][1]:.4f}, learned {le['rel_err'][1]:.4f}; steps/ray {pl['steps_per_ray'][1]:.1f} vs "
        f"{le['steps_per_ray'][1]:.1f}; work ratio {work[1] / work[0]:.3f}; error slope {le['err_slope']:.3f}")
    assert work[1] < 0.85 * work[0]
    assert -0.6 < le["err_slope"] < -0.4
