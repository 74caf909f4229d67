"""FP64 reference of the learned ray allocation (test infrastructure only).

The allocation network proposes, for every cell, a pdf over (band n, g-point g, octant o)
from which that cell's rays are drawn; each ray keeps the importance weight of Eq. 14 with
the probability it was drawn with, so the cell estimate stays unbiased for any positive pdf
(the same argument that lets Zhang's T_max pdf replace the cell's own emission pdf,
Sec. 2, Eqs. 13-14).

Model (one evaluation per cell and (n, g), eight octant logits each):
    features  f = [T_c / 1000 K, log10(1 + |grad T|_c), log10(kappa_P,c),
                   nu_n / 10^4 cm^-1, g_abscissa], standardised by stored (mu, s)
    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3), z = W4 h3 + b4
    octant logit of global octant o: z[o xor m_c], m_c = sign bits of grad T (x, y, z), so the
    network sees octants in a frame oriented by the local temperature gradient
    q_c = softmax over all (n, g, o) of z + log p_plain(n, g)   (the plain pdf as the prior:
          a network that outputs zero reproduces the plain allocation, and training learns
          corrections to it)
    p_c = (1 - eps) q_c + eps p_plain(n, g) / 8

Training objective, from rays i drawn with the plain pdf p0 (value Y_i = h_i / p0_i), for a
batch of cells c:
    M_c(p) = mean_{i in c} h_i^2 / (p0_i p_c(s_i))       (an unbiased estimate of E[Y^2] under p_c)
    C_c(p) = mean_{i in c} c_i p_c(s_i) / p0_i            (of the expected cost of a ray, c_i = 1
                                                          without costs)
    L(p)   = [sum_c M_c(p)] [sum_c C_c(p)] / ([sum_c M_c(p0)] [sum_c C_c(p0)]).
With R rays per cell the squared error of the field is sum_c Var_c / R and the work is
R sum_c C_c, so L is the work to reach a given RMS error relative to the plain allocation
(E[Y^2] and Var differ by the squared mean, which no unbiased allocation changes).  For one
cell the minimiser over pdfs is p_s proportional to sqrt(E[h^2 | s] / E[c | s])
(Cauchy-Schwarz).
"""
from __future__ import annotations

import numpy as np

SIGMA = 5.670374419e-8
N_IN, N_HID, N_OUT = 5, 64, 8
PARAM_SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
                ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_OUT, N_HID)), ("b4", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)   # 9224


def init_params(seed: int = 0) -> dict:
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in PARAM_SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[1])
            p[name] = rng.uniform(-lim, lim, shape)
        else:
            p[name] = np.zeros(shape)
    p["W4"] *= 0.1
    return p


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[n], dtype=np.float64).ravel() for n, _ in PARAM_SHAPES])


def unflatten(v: np.ndarray) -> dict:
    out, o = {}, 0
    for n, s in PARAM_SHAPES:
        k = int(np.prod(s))
        out[n] = np.asarray(v[o:o + k], dtype=np.float64).reshape(s)
        o += k
    return out


# ----------------------------------------------------------------------- features
def gradient_T(w) -> np.ndarray:
    """Central differences of T at the cell centres, shape [3, nx, ny, nz]: periodic in x and z;
    in y the walls enter as ghost values T_wall located on the wall faces."""
    nx, ny, nz = len(w.xf) - 1, len(w.yf) - 1, len(w.zf) - 1
    T = np.asarray(w.T, dtype=np.float64).reshape(nx, ny, nz)
    xc = 0.5 * (w.xf[:-1] + w.xf[1:])
    yc = 0.5 * (w.yf[:-1] + w.yf[1:])
    zc = 0.5 * (w.zf[:-1] + w.zf[1:])
    Lx, Lz = w.xf[-1] - w.xf[0], w.zf[-1] - w.zf[0]
    g = np.zeros((3, nx, ny, nz))
    xp, xm = np.roll(xc, -1), np.roll(xc, 1)
    dxp = np.where(np.arange(nx) == nx - 1, xp + Lx, xp)
    dxm = np.where(np.arange(nx) == 0, xm - Lx, xm)
    g[0] = (np.roll(T, -1, 0) - np.roll(T, 1, 0)) / (dxp - dxm)[:, None, None]
    zp, zm = np.roll(zc, -1), np.roll(zc, 1)
    dzp = np.where(np.arange(nz) == nz - 1, zp + Lz, zp)
    dzm = np.where(np.arange(nz) == 0, zm - Lz, zm)
    g[2] = (np.roll(T, -1, 2) - np.roll(T, 1, 2)) / (dzp - dzm)[None, None, :]
    Tg = np.concatenate([np.full((nx, 1, nz), w.T_walls[0]), T, np.full((nx, 1, nz), w.T_walls[1])], axis=1)
    yg = np.concatenate([[w.yf[0]], yc, [w.yf[-1]]])
    g[1] = (Tg[:, 2:, :] - Tg[:, :-2, :]) / (yg[2:] - yg[:-2])[None, :, None]
    return g


def planck_mean_tables(kd) -> np.ndarray:
    """Planck-mean absorption coefficient of every species at every table node,
    kP_s(T_t) = pi sum_{n,g} dnu w k^s_{n,g}(T_t) I_n(T_t) / (sigma T_t^4), shape [ns, nT]
    (0 at T = 0)."""
    Tg = kd.T0 + kd.dT * np.arange(kd.nT)
    num = np.pi * np.einsum("n,g,sngt,nt->st", kd.dnu, kd.wg, kd.k.astype(np.float64), kd.Ib)
    den = SIGMA * Tg ** 4
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def cell_features(w) -> np.ndarray:
    """Per-cell raw features [ncells, 3]: T/1000, log10(1 + |grad T|), log10(kappa_P) with
    kappa_P = sum_s x_s lerp(kP_s, T) (floored at 1e-30); and the gradient sign mask m_c."""
    from .closed_forms import table_lerp
    kd = w.kd
    g = gradient_T(w)
    gm = np.sqrt((g ** 2).sum(axis=0)).reshape(-1)
    kpt = planck_mean_tables(kd)
    kp = sum(np.asarray(w.X[s], dtype=np.float64) * table_lerp(kpt[s], kd.T0, kd.dT, w.T)
             for s in range(kd.ns))
    f = np.stack([np.asarray(w.T) / 1000.0, np.log10(1.0 + gm), np.log10(np.maximum(kp, 1e-30))], axis=1)
    m = ((g[0] < 0).astype(int) | ((g[1] < 0).astype(int) << 1) | ((g[2] < 0).astype(int) << 2)).reshape(-1)
    return f, m


def spectral_features(kd) -> np.ndarray:
    """Per (n, g) raw features [nb, ng, 2]: band centre / 10^4 cm^-1 and g abscissa."""
    nu = (kd.nu_lo + 0.5 * kd.dnu) / 1e4
    return np.stack(np.broadcast_arrays(nu[:, None], kd.gx[None, :]), axis=-1)


def assemble_inputs(fc, fs, mu, sd) -> np.ndarray:
    """Standardised network inputs [ncells, nb, ng, 5]."""
    nc, nb, ng = fc.shape[0], fs.shape[0], fs.shape[1]
    x = np.concatenate([np.broadcast_to(fc[:, None, None, :], (nc, nb, ng, 3)),
                        np.broadcast_to(fs[None], (nc, nb, ng, 2))], axis=-1)
    return (x - mu) / sd


# ------------------------------------------------------------------- network
def forward(p: dict, x: np.ndarray):
    """x [..., 5] -> logits [..., 8] and the activations needed by backward."""
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    a3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(a3, 0.0)
    z = h3 @ p["W4"].T + p["b4"]
    return z, (x, a1, h1, a2, h2, a3, h3)


def backward(p: dict, cache, dz: np.ndarray) -> dict:
    """Gradients of sum(dz * z) with respect to every parameter (chain rule, ReLU' = [a > 0])."""
    x, a1, h1, a2, h2, a3, h3 = cache
    X = x.reshape(-1, N_IN)
    H1, H2, H3 = h1.reshape(-1, N_HID), h2.reshape(-1, N_HID), h3.reshape(-1, N_HID)
    A1, A2, A3 = a1.reshape(-1, N_HID), a2.reshape(-1, N_HID), a3.reshape(-1, N_HID)
    D = dz.reshape(-1, N_OUT)
    g = {"W4": D.T @ H3, "b4": D.sum(0)}
    d3 = (D @ p["W4"]) * (A3 > 0)
    g["W3"], g["b3"] = d3.T @ H2, d3.sum(0)
    d2 = (d3 @ p["W3"]) * (A2 > 0)
    g["W2"], g["b2"] = d2.T @ H1, d2.sum(0)
    d1 = (d2 @ p["W2"]) * (A1 > 0)
    g["W1"], g["b1"] = d1.T @ X, d1.sum(0)
    return g


def octant_logits(z: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Global-octant logits: zg[c, n, g, o] = z[c, n, g, o xor m_c]."""
    idx = np.arange(8)[None, :] ^ np.asarray(m)[:, None]               # [nc, 8]
    return np.take_along_axis(z, idx[:, None, None, :], axis=-1)


def prior_logits(zg: np.ndarray, p_plain: np.ndarray) -> np.ndarray:
    """zg + log p_plain(n, g), the arguments of the allocation softmax."""
    with np.errstate(divide="ignore"):
        return zg + np.log(np.asarray(p_plain, dtype=np.float64))[None, :, :, None]


def cell_pdf(zg: np.ndarray, p_plain: np.ndarray, eps: float) -> np.ndarray:
    """p_c(n,g,o) = (1 - eps) softmax_{(n,g,o)}(zg_c + log p_plain(n,g)) + eps p_plain(n,g)/8,
    shape of zg."""
    nc = zg.shape[0]
    flat = prior_logits(zg, p_plain).reshape(nc, -1)
    e = np.exp(flat - flat.max(axis=1, keepdims=True))
    q = (e / e.sum(axis=1, keepdims=True)).reshape(zg.shape)
    return (1.0 - eps) * q + eps * (p_plain[None, :, :, None] / 8.0)


def allocation_loss(zg, p_plain, eps, cell_of, strata, h, p0, ray_cost=None):
    """L = [sum_c M_c(p)] [sum_c C_c(p)] / ([sum_c M_c(p0)] [sum_c C_c(p0)]) over the cells with
    samples (the cost factors are dropped without ray_cost).  Returns (L, dL/dzg)."""
    nc = zg.shape[0]
    shp = zg.shape
    flat = prior_logits(zg, p_plain).reshape(nc, -1)
    e = np.exp(flat - flat.max(axis=1, keepdims=True))
    sig = e / e.sum(axis=1, keepdims=True)
    pp = np.repeat(p_plain.reshape(-1), 8) / 8.0
    p = (1.0 - eps) * sig + eps * pp[None, :]
    c = np.ones(len(h)) if ray_cost is None else np.asarray(ray_cost, dtype=np.float64)
    cnt = np.bincount(cell_of, minlength=nc).astype(float)
    inv = np.where(cnt > 0, 1.0 / np.maximum(cnt, 1), 0.0)
    ps = p[cell_of, strata]
    num = h ** 2 / (p0 * ps)
    Mt = (np.bincount(cell_of, weights=num, minlength=nc) * inv).sum()
    M0 = (np.bincount(cell_of, weights=(h / p0) ** 2, minlength=nc) * inv).sum()
    if ray_cost is None:
        Ct = C0 = 1.0
    else:
        Ct = (np.bincount(cell_of, weights=c * ps / p0, minlength=nc) * inv).sum()
        C0 = (np.bincount(cell_of, weights=c, minlength=nc) * inv).sum()
    if not (M0 > 0 and C0 > 0):
        return 0.0, np.zeros(shp)
    L = Mt * Ct / (M0 * C0)
    G = np.zeros_like(p)                                                   # dL / dp_{c,s}
    np.add.at(G, (cell_of, strata), -num / ps * inv[cell_of] * Ct / (M0 * C0))
    if ray_cost is not None:
        np.add.at(G, (cell_of, strata), c / p0 * inv[cell_of] * Mt / (M0 * C0))
    dz = (1.0 - eps) * sig * (G - (G * sig).sum(axis=1, keepdims=True))
    return L, dz.reshape(shp)


def adam_step(v, g, m, s, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba, 2015) on flat parameter vectors; returns (v, m, s)."""
    m = b1 * m + (1 - b1) * g
    s = b2 * s + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    sh = s / (1 - b2 ** t)
    return v - lr * mh / (np.sqrt(sh) + eps), m, s
