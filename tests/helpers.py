"""Shared test helpers: oracle problems from set-ups, field comparison metrics."""
from __future__ import annotations

import numpy as np

import oracle
import rlb_inputs as ri


def problem(s: ri.Setup) -> oracle.Problem:
    return oracle.Problem(s.nx, s.ny, s.nz, s.batch, s.c_l, s.bc, s.inflow, s.tau, s.solid,
                          tau_cell=s.tau_cell, eta_s=s.eta_s, d_G=s.d_G, kappa=s.kappa)


def fluid_mask(s: ri.Setup) -> np.ndarray:
    if s.solid is None:
        return np.ones(s.cells, dtype=bool)
    return s.solid.reshape(-1) == 0


def field_err(gpu: np.ndarray, ref: np.ndarray, mask: np.ndarray) -> float:
    """max |gpu - ref| / max |ref| over the masked cells (norm-wise relative error:
    pointwise ratios are meaningless where a field crosses zero)."""
    g = gpu[..., mask]
    r = ref[..., mask]
    scale = np.abs(r).max()
    if scale == 0:
        return float(np.abs(g).max())
    return float(np.abs(g - r).max() / scale)


def oracle_fields(s: ri.Setup, steps: int):
    """(n, e, beta, sums, S) of the oracle after `steps` steps from the set-up."""
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    bad = oracle.run(p, S, steps)
    n, e, b, sums = oracle.moments(p, S)
    return n, e, b, sums, S, bad


def gpu_state(solver) -> np.ndarray:
    """Current GPU state as float64 [2][19][cells] (undeviated storages only)."""
    return solver.populations().double().cpu().numpy()
