"""Pins of the FP64 allocation-network reference: analytic backward against central finite
differences, the loss gradient against finite differences, and the loss minimiser against
its closed form p_s proportional to sqrt(E[h^2 | s])."""
import numpy as np
import pytest

from oracle import mlp
from paper_1810_00188_amd import inputs


def test_parameter_count():
    assert mlp.N_PARAMS == 9224


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1)
    for k in p:
        p[k] = p[k] + 0.05 * rng.normal(size=p[k].shape)   # nonzero biases
    x = rng.normal(size=(7, 3, mlp.N_IN))
    dz = rng.normal(size=(7, 3, mlp.N_OUT))
    z, cache = mlp.forward(p, x)
    g = mlp.flatten(mlp.backward(p, cache, dz))
    v = mlp.flatten(p)
    h = 1e-6
    idx = rng.choice(len(v), 300, replace=False)
    for q in idx:
        vp, vm = v.copy(), v.copy()
        vp[q] += h
        vm[q] -= h
        fp = np.sum(dz * mlp.forward(mlp.unflatten(vp), x)[0])
        fm = np.sum(dz * mlp.forward(mlp.unflatten(vm), x)[0])
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, g[q])


def _toy(nc=3, nb=2, ng=3, nray=40, seed=0):
    rng = np.random.default_rng(seed)
    p_plain = rng.dirichlet(np.ones(nb * ng)).reshape(nb, ng)
    zg = rng.normal(size=(nc, nb, ng, 8))
    cell_of = np.repeat(np.arange(nc), nray)
    strata = rng.integers(0, nb * ng * 8, nc * nray)
    p0 = np.repeat(p_plain.reshape(-1), 8)[strata] / 8
    h = rng.normal(size=nc * nray) * rng.uniform(0.1, 3, nc * nray)
    return zg, p_plain, cell_of, strata, h, p0


def test_loss_gradient_matches_finite_differences():
    zg, p_plain, cell_of, strata, h, p0 = _toy()
    L, dz = mlp.allocation_loss(zg, p_plain, 0.1, cell_of, strata, h, p0)
    hstep = 1e-6
    rng = np.random.default_rng(3)
    for q in rng.choice(zg.size, 60, replace=False):
        a, b = zg.copy().ravel(), zg.copy().ravel()
        a[q] += hstep
        b[q] -= hstep
        fd = (mlp.allocation_loss(a.reshape(zg.shape), p_plain, 0.1, cell_of, strata, h, p0)[0]
              - mlp.allocation_loss(b.reshape(zg.shape), p_plain, 0.1, cell_of, strata, h, p0)[0]) / (2 * hstep)
        assert abs(fd - dz.ravel()[q]) <= 1e-6 * max(1e-3, abs(fd))


def test_loss_minimiser_is_sqrt_second_moment():
    """With every stratum observed once per cell with weight h_s^2 (exact expectation), the
    minimiser over free logits (eps = 0) is p_s = sqrt(H_s) / sum sqrt(H)."""
    nb, ng = 2, 2
    S = nb * ng * 8
    rng = np.random.default_rng(5)
    H = rng.uniform(0.01, 4.0, S)
    p_plain = np.full((nb, ng), 1.0 / (nb * ng))
    strata = np.arange(S)
    p0 = np.full(S, 1.0 / S)
    h = np.sqrt(H) * p0              # the estimator's value h/p0 has square H
    cell_of = np.zeros(S, dtype=int)
    z = np.zeros((1, nb, ng, 8))
    m = np.zeros_like(z)
    s2 = np.zeros_like(z)
    for t in range(1, 6001):
        L, dz = mlp.allocation_loss(z, p_plain, 0.0, cell_of, strata, h, p0)
        v, m, s2 = mlp.adam_step(z.ravel(), dz.ravel(), m.ravel(), s2.ravel(), t, lr=0.02)
        z, m, s2 = v.reshape(z.shape), m.reshape(z.shape), s2.reshape(z.shape)
    p = mlp.cell_pdf(z, p_plain, 0.0).ravel()
    target = np.sqrt(H) / np.sqrt(H).sum()
    np.testing.assert_allclose(p, target, rtol=2e-3)


def test_cost_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(11)
    nc, nb, ng = 5, 3, 2
    zg = rng.normal(size=(nc, nb, ng, 8))
    p_plain = rng.uniform(0.2, 1.0, (nb, ng))
    p_plain /= p_plain.sum()
    cell_of = np.sort(rng.integers(0, nc, 40))
    strata = rng.integers(0, nb * ng * 8, 40)
    h = rng.normal(size=40)
    p0 = rng.uniform(0.01, 0.2, 40)
    cost = rng.uniform(1.0, 30.0, 40)
    L, dz = mlp.allocation_loss(zg, p_plain, 0.1, cell_of, strata, h, p0, ray_cost=cost)
    v = zg.ravel()
    for q in rng.choice(v.size, 60, replace=False):
        a, b = v.copy(), v.copy()
        a[q] += 1e-6
        b[q] -= 1e-6
        fd = (mlp.allocation_loss(a.reshape(zg.shape), p_plain, 0.1, cell_of, strata, h, p0, ray_cost=cost)[0]
              - mlp.allocation_loss(b.reshape(zg.shape), p_plain, 0.1, cell_of, strata, h, p0, ray_cost=cost)[0]) / 2e-6
        assert abs(fd - dz.ravel()[q]) <= 1e-6 * (1 + abs(fd))
    # rays drawn with the plain pdf and p = p_plain / 8 (eps = 1): the cost factor is exactly 1
    pr = np.repeat(p_plain.ravel(), 8)[strata] / 8.0
    L1, _ = mlp.allocation_loss(zg, p_plain, 1.0, cell_of, strata, h, pr, ray_cost=cost)
    L2, _ = mlp.allocation_loss(zg, p_plain, 1.0, cell_of, strata, h, pr)
    assert abs(L1 - L2) < 1e-12 * abs(L2)


def test_cost_loss_minimiser_is_work_normalised():
    """With every stratum observed once per cell (exact expectations H_s and costs c_s), the
    minimiser of second moment x expected cost is p_s = sqrt(H_s / c_s) / sum sqrt(H / c)
    (Cauchy-Schwarz)."""
    nb, ng = 2, 2
    S = nb * ng * 8
    rng = np.random.default_rng(6)
    H = rng.uniform(0.01, 4.0, S)
    cs = rng.uniform(1.0, 20.0, S)
    p_plain = np.full((nb, ng), 1.0 / (nb * ng))
    strata = np.arange(S)
    p0 = np.full(S, 1.0 / S)
    h = np.sqrt(H) * p0
    cell_of = np.zeros(S, dtype=int)
    z = np.zeros((1, nb, ng, 8))
    m = np.zeros_like(z)
    s2 = np.zeros_like(z)
    for t in range(1, 8001):
        L, dz = mlp.allocation_loss(z, p_plain, 0.0, cell_of, strata, h, p0, ray_cost=cs)
        v, m, s2 = mlp.adam_step(z.ravel(), dz.ravel(), m.ravel(), s2.ravel(), t, lr=0.02)
        z, m, s2 = v.reshape(z.shape), m.reshape(z.shape), s2.reshape(z.shape)
    p = mlp.cell_pdf(z, p_plain, 0.0).ravel()
    target = np.sqrt(H / cs) / np.sqrt(H / cs).sum()
    np.testing.assert_allclose(p, target, rtol=3e-3)


def test_batch_objective_is_invariant_to_copies():
    """The objective is a ratio of batch totals: a batch of identical copies of one cell has
    the cell's value, and each copy receives the cell's gradient divided by the number of
    copies."""
    rng = np.random.default_rng(13)
    nb, ng, k = 2, 3, 4
    zg1 = rng.normal(size=(1, nb, ng, 8))
    p_plain = rng.uniform(0.2, 1.0, (nb, ng))
    p_plain /= p_plain.sum()
    strata = rng.integers(0, nb * ng * 8, 12)
    h = rng.normal(size=12)
    p0 = rng.uniform(0.01, 0.2, 12)
    cost = rng.uniform(1.0, 30.0, 12)
    L1, d1 = mlp.allocation_loss(zg1, p_plain, 0.1, np.zeros(12, int), strata, h, p0, ray_cost=cost)
    Lk, dk = mlp.allocation_loss(np.repeat(zg1, k, axis=0), p_plain, 0.1, np.repeat(np.arange(k), 12),
                                 np.tile(strata, k), np.tile(h, k), np.tile(p0, k), ray_cost=np.tile(cost, k))
    assert abs(Lk - L1) < 1e-13 * abs(L1)
    np.testing.assert_allclose(dk, np.repeat(d1 / k, k, axis=0), rtol=1e-12, atol=1e-18)


def test_octant_frame_and_pdf_normalisation():
    rng = np.random.default_rng(2)
    z = rng.normal(size=(4, 2, 3, 8))
    m = np.array([0, 1, 5, 7])
    zg = mlp.octant_logits(z, m)
    for c in range(4):
        for o in range(8):
            assert np.array_equal(zg[c, :, :, o], z[c, :, :, o ^ m[c]])
    p = mlp.cell_pdf(zg, np.full((2, 3), 1 / 6), 0.2)
    np.testing.assert_allclose(p.reshape(4, -1).sum(axis=1), 1.0, rtol=1e-14)
    assert np.all(p >= 0.2 / 6 / 8 - 1e-18)


def test_features_and_gradient():
    w = inputs.channel(nx=6, ny=5, nz=4, nb=3, ng=2, amp=0.1).replace(T_walls=(300.0, 500.0))
    g = mlp.gradient_T(w)
    # a linear field in x (periodic central difference of a linear profile away from the seam)
    T = np.broadcast_to((500.0 + 10.0 * np.arange(6))[:, None, None], (6, 5, 4)).reshape(-1)
    gl = mlp.gradient_T(w.replace(T=T))
    dx = w.xf[1] - w.xf[0]
    np.testing.assert_allclose(gl[0][1:-1], 10.0 / dx, rtol=1e-12)
    fc, m = mlp.cell_features(w)
    assert fc.shape == (w.ncells, 3) and m.shape == (w.ncells,)
    kpt = mlp.planck_mean_tables(w.kd)
    assert kpt.shape == (1, w.kd.nT)
    assert kpt[0, 100] == pytest.approx(10.0 / 0.1, rel=1e-6)   # table scaled to 10 m^-1 at x = 0.1
    assert g.shape == (3, 6, 5, 4)


def test_zero_network_output_is_the_plain_allocation():
    """The allocation softmax runs over the network's logits plus log p_plain(n, g): logits
    that are equal for every stratum give exactly the plain pdf p_plain(n, g) / 8 for any
    mixture weight, and the training objective of rays drawn from it is exactly 1."""
    rng = np.random.default_rng(2)
    nb, ng, nc = 4, 3, 6
    p_plain = rng.uniform(0.01, 1.0, (nb, ng))
    p_plain /= p_plain.sum()
    for eps in (0.0, 0.3, 1.0):
        zg = np.full((nc, nb, ng, 8), rng.normal())
        p = mlp.cell_pdf(zg, p_plain, eps)
        np.testing.assert_allclose(p, np.broadcast_to(p_plain[None, :, :, None] / 8, p.shape), rtol=1e-14)
    strata = rng.integers(0, nb * ng * 8, 50)
    p0 = np.repeat(p_plain.ravel(), 8)[strata] / 8.0
    cell_of = np.sort(rng.integers(0, nc, 50))
    L, dz = mlp.allocation_loss(np.zeros((nc, nb, ng, 8)), p_plain, 0.1, cell_of, strata, rng.normal(size=50), p0,
                                ray_cost=rng.uniform(1, 5, 50))
    assert abs(L - 1.0) < 1e-13
