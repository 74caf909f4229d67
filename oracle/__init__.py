"""CPU oracle of the emission-based reciprocal Monte Carlo (ERMC) radiative heat source.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``; the product path (the HIP library and its binding) never
imports, links or executes anything here, and this package never imports the product.

* ``rmc_oracle.c`` -- plain FP64 C: Philox4x32-10, table interpolation, the T_max spectral
  pdf, ray sampling, the Algorithm-1 march and the per-cell estimate (see its header for the
  paper passages and the readings taken where the paper is silent).
* ``closed_forms`` -- exact expectations the Monte Carlo estimate must reproduce
  (grey isothermal slab, layered 1-D media, optically thin limit).
* ``mlp`` -- FP64 reference of the ray-allocation network (forward, backward, Adam).

The shared library is compiled from ``rmc_oracle.c`` with gcc (``build()``); IEEE FP64,
no fast-math, no FMA contraction.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rmc_oracle.c")
LIB = os.path.join(HERE, "librmc_oracle.so")

GCC_CMD = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", SRC, "-o", LIB, "-lm"]

ERRORS = {0: "ok", 1: "invalid argument", 3: "temperature outside the table range",
          4: "unsupported"}


def build() -> str:
    """Compile the oracle shared library (always recompiles)."""
    subprocess.run(GCC_CMD, check=True)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        L.orc_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_plain_pdf.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_trace_cells.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_divergence.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int]
        L.orc_march.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.orc_march_mg.argtypes = L.orc_march.argtypes
        L.orc_wall_flux.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_level_count.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_level_count.restype = C.c_int
        L.orc_coarse_fields.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("xf", C.c_void_p), ("yf", C.c_void_p), ("zf", C.c_void_p),
                ("T", C.c_void_p), ("ns", C.c_int), ("X", C.c_void_p),
                ("Tw", C.c_double * 2), ("epsw", C.c_double * 2),
                ("nb", C.c_int), ("ng", C.c_int), ("nT", C.c_int),
                ("T0", C.c_double), ("dT", C.c_double),
                ("dnu", C.c_void_p), ("wg", C.c_void_p), ("k", C.c_void_p), ("Ib", C.c_void_p),
                ("R", C.c_int), ("seed", C.c_uint64), ("snap", C.c_uint32),
                ("tol", C.c_double), ("max_steps", C.c_int),
                ("q_cell", C.c_void_p), ("mix_eps", C.c_double),
                ("mg_levels", C.c_int), ("mg_steps", C.c_int),
                ("closed", C.c_int), ("Tx", C.c_double * 2), ("epsx", C.c_double * 2),
                ("Tz", C.c_double * 2), ("epsz", C.c_double * 2)]


class _MarchOut(C.Structure):
    _fields_ = [("acc", C.c_double), ("absacc", C.c_double), ("steps", C.c_int), ("end", C.c_int),
                ("wacc", C.c_double), ("wall", C.c_int), ("wface", C.c_int)]


RAY_DTYPE = np.dtype([("Y", "f8"), ("absY", "f8"), ("p", "f8"), ("n", "i4"), ("g", "i4"),
                      ("o", "i4"), ("k", "i4"), ("steps", "i4"), ("end", "i4")])


class OracleError(RuntimeError):
    pass


def _check(code):
    if code != 0:
        raise OracleError(ERRORS.get(code, f"error {code}"))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """A workload (``paper_1810_00188_amd.inputs.Workload``-like object) in oracle form.

    Any object with the attributes xf, yf, zf, T, X, kd, T_walls, eps_walls, R, seed, snap,
    tol, max_steps works; ``q_cell`` ([ncells, nb, ng, 8]) switches to a per-cell
    allocation pdf mixed with ``mix_eps`` of the plain one.  ``mg_levels`` / ``mg_steps``
    (default: the workload's, else the DNS grid alone) select the multigrid march.
    """

    def __init__(self, w, q_cell: Optional[np.ndarray] = None, mix_eps: float = 0.0,
                 mg_levels: Optional[int] = None, mg_steps: Optional[int] = None):
        kd = w.kd
        self._keep = dict(xf=_f64(w.xf), yf=_f64(w.yf), zf=_f64(w.zf), T=_f64(w.T),
                          X=_f64(np.atleast_2d(w.X)), dnu=_f64(kd.dnu), wg=_f64(kd.wg),
                          k=_f64(kd.k), Ib=_f64(kd.Ib))
        if q_cell is not None:
            self._keep["q"] = _f64(q_cell)
        K = self._keep
        s = _Problem()
        s.nx, s.ny, s.nz = len(K["xf"]) - 1, len(K["yf"]) - 1, len(K["zf"]) - 1
        s.xf, s.yf, s.zf = K["xf"].ctypes.data, K["yf"].ctypes.data, K["zf"].ctypes.data
        s.T = K["T"].ctypes.data
        s.ns = K["X"].shape[0]
        s.X = K["X"].ctypes.data
        s.Tw[0], s.Tw[1] = float(w.T_walls[0]), float(w.T_walls[1])
        s.epsw[0], s.epsw[1] = float(w.eps_walls[0]), float(w.eps_walls[1])
        s.nb, s.ng, s.nT = kd.k.shape[1], kd.k.shape[2], kd.k.shape[3]
        s.T0, s.dT = float(kd.T0), float(kd.dT)
        s.dnu, s.wg, s.k, s.Ib = (K["dnu"].ctypes.data, K["wg"].ctypes.data,
                                  K["k"].ctypes.data, K["Ib"].ctypes.data)
        s.R, s.seed, s.snap = int(w.R), int(w.seed), int(w.snap)
        s.tol, s.max_steps = float(w.tol), int(w.max_steps)
        s.q_cell = K["q"].ctypes.data if q_cell is not None else None
        s.mix_eps = float(mix_eps)
        s.mg_levels = int(getattr(w, "mg_levels", 1) if mg_levels is None else mg_levels)
        s.mg_steps = int(getattr(w, "mg_steps", 5) if mg_steps is None else mg_steps)
        s.closed = int(bool(getattr(w, "closed", False)))
        if s.closed:
            for q in range(2):
                s.Tx[q], s.epsx[q] = float(w.T_walls_x[q]), float(w.eps_walls_x[q])
                s.Tz[q], s.epsz[q] = float(w.T_walls_z[q]), float(w.eps_walls_z[q])
        self.s = s
        self.nx, self.ny, self.nz = s.nx, s.ny, s.nz
        self.ncells = s.nx * s.ny * s.nz
        self.R = s.R
        self.nb, self.ng = s.nb, s.ng

    @property
    def ptr(self):
        return C.byref(self.s)


def philox(ctr, key):
    """Philox4x32-10 block: four 32-bit counter words, two key words -> four words."""
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return tuple(int(x) for x in o)


@dataclass
class PlainPdf:
    p: np.ndarray        # [nb, ng]
    cdf_b: np.ndarray    # [nb]
    cdf_g: np.ndarray    # [nb, ng]
    Tmax: float


def plain_pdf(prob: Problem) -> PlainPdf:
    p = np.zeros((prob.nb, prob.ng))
    cb = np.zeros(prob.nb)
    cg = np.zeros((prob.nb, prob.ng))
    tm = C.c_double()
    _check(lib().orc_plain_pdf(prob.ptr, p.ctypes.data, cb.ctypes.data, cg.ctypes.data,
                               C.addressof(tm)))
    return PlainPdf(p, cb, cg, tm.value)


def trace_cells(prob: Problem, cells) -> np.ndarray:
    """Per-ray records (RAY_DTYPE) of all R rays of each listed cell, shape [len(cells), R]."""
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((len(cells), prob.R), dtype=RAY_DTYPE)
    _check(lib().orc_trace_cells(prob.ptr, len(cells), cells.ctypes.data, out.ctypes.data))
    return out


def divergence(prob: Problem, cells=None, nthreads: int = 0):
    """(divq, stderr, total ray-cell steps) for all cells (natural order) or a cell list."""
    if cells is not None:
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        n = len(cells)
    else:
        n = prob.ncells
    dq = np.zeros(n)
    se = np.zeros(n)
    st = C.c_int64()
    _check(lib().orc_divergence(prob.ptr, n if cells is not None else 0,
                                cells.ctypes.data if cells is not None else None,
                                dq.ctypes.data, se.ctypes.data, C.addressof(st), int(nthreads)))
    return dq, se, st.value


def wall_flux(prob: Problem) -> np.ndarray:
    """Net radiative flux from the gas into every wall face element [W m^-2] (black walls, one
    grid), flat: x0 [ny*nz], x1, y0 [nx*nz], y1, z0 [nx*ny], z1 (see split_walls)."""
    q = np.zeros(2 * (prob.ny * prob.nz + prob.nx * prob.nz + prob.nx * prob.ny))
    _check(lib().orc_wall_flux(prob.ptr, q.ctypes.data))
    return q


def split_walls(prob: Problem, q) -> dict:
    """The six wall arrays of a flat wall-flux vector: x0, x1 [ny, nz], y0, y1 [nx, nz], z0, z1 [nx, ny]."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    sizes = [ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny]
    shapes = [(ny, nz), (ny, nz), (nx, nz), (nx, nz), (nx, ny), (nx, ny)]
    o = np.concatenate([[0], np.cumsum(sizes)])
    return {k: np.asarray(q)[o[u]:o[u + 1]].reshape(shapes[u]) for u, k in enumerate(("x0", "x1", "y0", "y1", "z0", "z1"))}


def march(prob: Problem, cell_ijk, n: int, g: int, d, record: int = 0, multigrid: bool = False):
    """March one ray of band n, g-point g from the centre of cell (i, j, k) along d.

    Returns dict(acc, absacc, steps, end, wall, wface, wacc[, cells, ds]) -- the accumulated
    sum tau alpha (I_c - I_j) (+ wall and residual terms) before the ray weight; wall / wface /
    wacc: the black wall (0..5: x0, x1, y0, y1, z0, z1; -1 none) that ended the ray, the face
    element it reached there and the wall term of acc.  With
    ``multigrid`` the ray takes the multigrid march of the problem's mg_levels / mg_steps and
    the recorded cells are (level, natural index within that level) pairs."""
    d = _f64(d)
    m = _MarchOut()
    rc = np.zeros(max(record, 1), dtype=np.int64)
    rd = np.zeros(max(record, 1))
    i, j, k = (int(x) for x in cell_ijk)
    fn = lib().orc_march_mg if multigrid else lib().orc_march
    _check(fn(prob.ptr, i, j, k, int(n), int(g), d.ctypes.data, C.addressof(m),
              rc.ctypes.data if record else None, rd.ctypes.data if record else None, int(record)))
    out = dict(acc=m.acc, absacc=m.absacc, steps=m.steps, end=m.end, wall=m.wall, wface=m.wface, wacc=m.wacc)
    if record:
        cells = rc[:min(m.steps, record)]
        if multigrid:
            out["level"] = (cells >> 48).astype(np.int64)
            cells = cells & ((1 << 48) - 1)
        out["cells"] = cells
        out["ds"] = rd[:min(m.steps, record)]
    return out


def level_count(nx: int, ny: int, nz: int) -> int:
    """Number of overlaid grid levels the multigrid march can use on an nx x ny x nz grid."""
    return int(lib().orc_level_count(int(nx), int(ny), int(nz)))


def coarse_fields(prob: Problem, level: int):
    """(T, X) of grid level ``level``: [ncells_L] and [ns, ncells_L], natural order of the level."""
    nl = (prob.nx >> level) * (prob.ny >> level) * (prob.nz >> level)
    T = np.zeros(nl)
    X = np.zeros((prob.s.ns, nl))
    _check(lib().orc_coarse_fields(prob.ptr, int(level), T.ctypes.data, X.ctypes.data))
    return T, X


def max_threads() -> int:
    return int(lib().orc_max_threads())
