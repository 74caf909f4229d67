"""Trained ray-allocation networks, one file per workload generator.

Each ``<workload>.npz`` holds what rmc_set_allocator takes for that workload's tables --
``params`` (float32[RMC_MLP_PARAMS], the layout of rmc_set_allocator), the input
standardisation ``mu`` / ``sd`` (float32[5]) -- the defensive mixture weight ``mix_eps`` it was
trained with, and ``info``, a JSON text describing the training run (fields, rays, Adam steps,
final loss).  Written by ``bench.py --learned <workload> --save-allocator``; read without
pickles (``numpy.load(..., allow_pickle=False)``).
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def path_of(workload: str) -> str:
    return os.path.join(HERE, f"{workload}.npz")


def save(workload: str, params, mu, sd, mix_eps: float, info: dict) -> str:
    p = path_of(workload)
    np.savez(p, params=np.ascontiguousarray(params, dtype=np.float32),
             mu=np.ascontiguousarray(mu, dtype=np.float32), sd=np.ascontiguousarray(sd, dtype=np.float32),
             mix_eps=np.float64(mix_eps), info=np.array(json.dumps(info, sort_keys=True)))
    return p


def load(workload: str) -> dict:
    p = path_of(workload)
    if not os.path.exists(p):
        raise FileNotFoundError(f"no trained allocation network for workload {workload!r} ({p})")
    with np.load(p, allow_pickle=False) as z:
        return {"params": z["params"].copy(), "mu": z["mu"].copy(), "sd": z["sd"].copy(),
                "mix_eps": float(z["mix_eps"]), "info": json.loads(str(z["info"]))}
