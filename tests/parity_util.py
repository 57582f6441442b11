"""Helpers for GPU-vs-oracle parity tests (test infrastructure)."""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

KB, DA = 1.380649e-23, 1.66053906892e-27


def make_pair(fields, ions, srcs, op, cap, *, precision=0, seed=7, fp32_tables=False, timing=False):
    from oracle.binding import OracleSim
    from paper_2609_31258_amd import mucite
    g = mucite.Sim(seed=seed, pack_capacity=cap, precision=precision, fp32_tables=fp32_tables, timing=timing)
    g.setup(fields, ions, srcs, op)
    o = OracleSim(seed)
    o.setup(fields, ions, srcs, op)
    return g, o


def by_id(p: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    order = np.argsort(p["id"], kind="stable")
    return {k: v[order] for k, v in p.items()}


def step_errors(gpu: Dict[str, np.ndarray], orc: Dict[str, np.ndarray], dr: float, a_g: float,
                h_prev: np.ndarray) -> Dict[str, object]:
    """Per-pack single-step acceptance of the GPU state against the oracle:
    |dx| <= 1e-6 (|x| + dr), |dv| <= 1e-6 (|v| + a_g), |dE_int| <= 1e-6 E_int,
    |dH| <= 1e-6 (H + k dt), identical status."""
    a, b = by_id(gpu), by_id(orc)
    assert np.array_equal(a["id"], b["id"])
    X = lambda p: np.stack([p["x"], p["y"], p["z"]], 1)
    V = lambda p: np.stack([p["vx"], p["vy"], p["vz"]], 1)
    dx = np.linalg.norm(X(a) - X(b), axis=1) / (np.linalg.norm(X(b), axis=1) + dr)
    dv = np.linalg.norm(V(a) - V(b), axis=1) / (np.linalg.norm(V(b), axis=1) + a_g)
    de = np.abs(a["e_int"] - b["e_int"]) / np.maximum(np.abs(b["e_int"]), 1e-300)
    kdt = np.abs(b["h"] - h_prev)
    dh = np.abs(a["h"] - b["h"]) / np.maximum(np.abs(b["h"]) + kdt, 1e-300)
    dh[(a["h"] == b["h"])] = 0.0
    same = a["status"] == b["status"]
    ok = same & (dx <= 1e-6) & (dv <= 1e-6) & (de <= 1e-6) & (dh <= 1e-6)
    return dict(ok=ok, same_status=same, dx=dx, dv=dv, de=de, dh=dh, n=len(ok),
                max_dx=float(dx.max(initial=0)), max_dv=float(dv.max(initial=0)),
                max_de=float(de.max(initial=0)), max_dh=float(dh.max(initial=0)))


def thermal_speed(t_gas=300.0, m_gas_da=28.0134) -> float:
    return math.sqrt(KB * t_gas / (m_gas_da * DA))


def frac_bound(fa, fb, na, nb):
    """4-sigma bound on a difference of two weighted fractions."""
    f = 0.5 * (fa + fb)
    return 4.0 * math.sqrt(max(f * (1 - f), 1e-12) * (1.0 / max(na, 1) + 1.0 / max(nb, 1)))
