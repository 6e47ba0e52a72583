"""FP64 CPU oracle for the relativistic lattice Boltzmann step (TEST INFRASTRUCTURE).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_0912_2913_amd``) and never imports it; the two meet only through the
seeded input generators in ``rlb_inputs``.

Contents:
  * ``liboracle_rlb.so`` (built from ``rlb_oracle.cpp``): the D3Q19 two-population
    scheme of the paper (eqs. lbe1/lbe2, equil1s/equil2as/equil2bs, the macroscopic
    constraints closed by e = 3P), plain single-threaded loops, templated on the
    scalar so that complex-step derivatives are exact references.
  * ``d1q3``: an independent lumped one-dimensional form of the same scheme.
  * ``riemann``: the exact ideal Riemann solution for P = e/3 (convergence target).

Layout of every array passed here: populations ``[2][19][cells]`` (f then g; the
g-only calls take ``[19][cells]``), fields ``[cells]``, velocities ``[3][cells]``;
``cells = batch*nz*ny*nx`` with x fastest.  Boundary codes: 0 periodic, 1 outflow
(zero-gradient copy), 2 inflow (face held at the inflow equilibrium).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_rlb.so")
_lib = None

PERIODIC, OUTFLOW, INFLOW = 0, 1, 2
Q = 19

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_lp = ctypes.POINTER(ctypes.c_long)


def lib():
    """Load (building first if absent or stale) the oracle library.  The
    environment variable RLB_ORACLE_LIB selects another build of the same
    source (the mutation tests load deliberately broken copies that way)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("RLB_ORACLE_LIB")
    if not path:
        path = _LIB_PATH
        src = os.path.join(_HERE, "rlb_oracle.cpp")
        if (not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
    L = ctypes.CDLL(path)
    L.ora_lattice.argtypes = [_ip, _dp, _ip]
    L.ora_equilibria.argtypes = [ctypes.c_double, ctypes.c_double, _dp, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp]
    L.ora_invert.argtypes = [ctypes.c_double, ctypes.c_double, _dp, ctypes.c_double, _dp]
    L.ora_invert.restype = ctypes.c_int
    L.ora_collide.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp,
                              _dp]
    L.ora_collide.restype = ctypes.c_int
    common = [_ip, ctypes.c_double, _ip, _dp, _u8p]
    L.ora_init.argtypes = common + [ctypes.c_double, _dp, _dp, _dp, _dp]
    rxp = ctypes.POINTER(Relax)
    L.ora_run.argtypes = common + [rxp, _dp, ctypes.c_int]
    L.ora_run.restype = ctypes.c_long
    L.ora_run_tracked.argtypes = common + [rxp, _dp, ctypes.c_int, _u8p, _lp]
    L.ora_run_tracked.restype = ctypes.c_long
    L.ora_run_g.argtypes = common + [rxp, _dp, ctypes.c_int]
    L.ora_run_g.restype = ctypes.c_long
    L.ora_update_cells.argtypes = common + [rxp, _dp, ctypes.c_long, _lp, _dp]
    L.ora_moments.argtypes = [_ip, ctypes.c_double, ctypes.c_double, _u8p, _dp, _dp, _dp, _dp,
                              _dp]
    L.ora_adjoint_step.argtypes = common + [rxp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_adjoint_step.restype = ctypes.c_int
    L.ora_transport.argtypes = [_ip, ctypes.c_double, _u8p, _dp, rxp, _dp, _dp, _dp, _dp]
    L.ora_transport.restype = ctypes.c_int
    L.ora_moments_adjoint.argtypes = [_ip, ctypes.c_double, ctypes.c_double, _u8p, _dp, _dp, _dp,
                                      _dp]
    L.ora_init_adjoint.argtypes = common + [ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_loss.argtypes = common + [rxp, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp]
    L.ora_loss.restype = ctypes.c_double
    L.ora_loss_cs.argtypes = common + [rxp, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp,
                                       _dp, _dp, _dp, _dp, _dp, _dp]
    L.ora_loss_cs.restype = ctypes.c_double
    L.ora_gradient.argtypes = common + [rxp, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp,
                                        _dp, _dp, _dp, _dp, _dp]
    L.ora_gradient.restype = ctypes.c_double
    _lib = L
    return L


def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> Optional[np.ndarray]:
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Relax(ctypes.Structure):
    """Relaxation source of a run (mirrors the oracle's OraRelax)."""

    _fields_ = [("tau", _dp), ("tau_cell", _dp), ("eta_s", ctypes.c_double),
                ("d_G", ctypes.c_double), ("kappa", ctypes.c_double)]


@dataclass
class Problem:
    """A lattice problem in the oracle's terms (all host data, FP64)."""

    nx: int
    ny: int
    nz: int
    batch: int = 1
    c_l: float = 1.0
    bc: Sequence[Sequence[int]] = ((0, 0), (0, 0), (0, 0))
    inflow: Sequence[float] = (1.0, 1.0, 0.0, 0.0, 0.0)  # n, e, beta_x, beta_y, beta_z
    tau: Sequence[float] = (0.6,)
    solid: Optional[np.ndarray] = None  # uint8 [cells]
    tau_cell: Optional[np.ndarray] = None  # [cells]: per-cell relaxation times
    eta_s: float = 0.0  # > 0: hold eta/s fixed (tau from the local state, f+g runs)
    d_G: float = 16.0  # degeneracy in n_eq = d_G T^3 / pi^2
    kappa: float = 1.0 / 3.0  # equation of state P = kappa e

    @property
    def cells(self) -> int:
        return self.batch * self.nz * self.ny * self.nx

    def _args(self):
        dims = np.array([self.nx, self.ny, self.nz, self.batch], dtype=np.int32)
        bc = np.array([v for ax in self.bc for v in ax], dtype=np.int32)
        inflow = np.array(self.inflow, dtype=np.float64)
        solid = None
        if self.solid is not None:
            solid = np.ascontiguousarray(self.solid.reshape(-1).astype(np.uint8))
            assert solid.size == self.cells
        tau = np.array(self.tau, dtype=np.float64).reshape(-1)
        if tau.size == 1 and self.batch > 1:
            tau = np.full(self.batch, tau[0])
        assert tau.size == self.batch
        tc = None
        if self.tau_cell is not None:
            tc = np.ascontiguousarray(np.asarray(self.tau_cell, dtype=np.float64).reshape(-1))
            assert tc.size == self.cells
        rx = Relax(tau.ctypes.data_as(_dp), tc.ctypes.data_as(_dp) if tc is not None else None,
                   float(self.eta_s), float(self.d_G), float(self.kappa))
        self._keep = (dims, bc, inflow, solid, tau, tc, rx)
        return (dims.ctypes.data_as(_ip), ctypes.c_double(self.c_l), bc.ctypes.data_as(_ip),
                inflow.ctypes.data_as(_dp),
                solid.ctypes.data_as(_u8p) if solid is not None else None), ctypes.byref(rx)


def lattice():
    """(e[19][3], w[19], opp[19]) as the oracle defines them."""
    e = np.zeros((Q, 3), np.int32)
    w = np.zeros(Q)
    o = np.zeros(Q, np.int32)
    lib().ora_lattice(e.ctypes.data_as(_ip), _d(w), o.ctypes.data_as(_ip))
    return e, w, o


def equilibria(n, eps, beta, c_l, kappa=1.0 / 3.0):
    """(f^eq, g^eq); kappa = 1/3 uses eqs. equil1s/equil2as/equil2bs, any other
    kappa eqs. equil1/equil2a/equil2b with P = kappa e."""
    feq = np.zeros(Q)
    geq = np.zeros(Q)
    b = _f64(beta)
    lib().ora_equilibria(float(n), float(eps), _d(b), float(c_l), float(kappa), _d(feq), _d(geq))
    return feq, geq


def invert(N, E, M, kappa=1.0 / 3.0):
    out = np.zeros(5)
    m = _f64(M)
    ok = lib().ora_invert(float(N), float(E), _d(m), float(kappa), _d(out))
    return out[0], out[1], out[2:5].copy(), bool(ok)


def collide(pf, pg, tau, c_l, kappa=1.0 / 3.0):
    pf, pg = _f64(pf), _f64(pg)
    of = np.zeros(Q)
    og = np.zeros(Q)
    ok = lib().ora_collide(_d(pf), _d(pg), float(tau), float(c_l), float(kappa), _d(of), _d(og))
    return of, og, bool(ok)


def init(p: Problem, n0, e0, beta0) -> np.ndarray:
    """S_0 ([2][19][cells]) from initial fields n0, e0 [cells], beta0 [3][cells]."""
    args, _ = p._args()
    n0, e0, beta0 = _f64(n0).reshape(-1), _f64(e0).reshape(-1), _f64(beta0).reshape(3, -1)
    S = np.zeros((2, Q, p.cells))
    lib().ora_init(*args, float(p.kappa), _d(n0), _d(e0), _d(np.ascontiguousarray(beta0)), _d(S))
    return S


def run(p: Problem, S: np.ndarray, nsteps: int) -> int:
    """Advance S ([2][19][cells], in place) by nsteps; returns the unphysical-update count."""
    if p.eta_s > 0 and p.kappa != 1.0 / 3.0:
        raise ValueError("the eta/s rule is defined for e = 3P matter (kappa = 1/3)")
    args, rx = p._args()
    assert S.shape == (2, Q, p.cells) and S.dtype == np.float64 and S.flags.c_contiguous
    return int(lib().ora_run(*args, rx, _d(S), int(nsteps)))


def run_tracked(p: Problem, S: np.ndarray, nsteps: int, mark: Optional[np.ndarray] = None):
    """run() with a record of f-positivity (the discussion section's bound
    c_i.u > -c_l^2/3 for f^eq_i > 0).  Returns (unphysical updates, updates
    whose f^eq broke the bound, mark): mark[cells] = 1 where the final f
    depends on such an update (the update itself or, through the pulls, an
    earlier one upstream).  Pass the mark of an earlier run to continue it."""
    if p.eta_s > 0 and p.kappa != 1.0 / 3.0:
        raise ValueError("the eta/s rule is defined for e = 3P matter (kappa = 1/3)")
    args, rx = p._args()
    assert S.shape == (2, Q, p.cells) and S.dtype == np.float64 and S.flags.c_contiguous
    m = np.zeros(p.cells, np.uint8) if mark is None else np.ascontiguousarray(mark, np.uint8).copy()
    lost = ctypes.c_long(0)
    bad = lib().ora_run_tracked(*args, rx, _d(S), int(nsteps), m.ctypes.data_as(_u8p),
                                ctypes.byref(lost))
    return int(bad), int(lost.value), m.astype(bool)


def run_g(p: Problem, Sg: np.ndarray, nsteps: int) -> int:
    if p.eta_s > 0:
        raise ValueError("holding eta/s needs the f population: use run()")
    args, rx = p._args()
    assert Sg.shape == (Q, p.cells) and Sg.flags.c_contiguous
    return int(lib().ora_run_g(*args, rx, _d(Sg), int(nsteps)))


def update_cells(p: Problem, S: np.ndarray, idx) -> np.ndarray:
    """One step evaluated at the given linear cell indices: returns [k][38] (f then g)."""
    args, rx = p._args()
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.zeros((idx.size, 2 * Q))
    lib().ora_update_cells(*args, rx, _d(S), ctypes.c_long(idx.size),
                           idx.ctypes.data_as(_lp), _d(out))
    return out


def moments(p: Problem, S: np.ndarray):
    """(n, e, beta[3][cells], sums[batch][5]) of a stored state."""
    dims = np.array([p.nx, p.ny, p.nz, p.batch], dtype=np.int32)
    solid = None if p.solid is None else np.ascontiguousarray(p.solid.reshape(-1).astype(np.uint8))
    n = np.zeros(p.cells)
    e = np.zeros(p.cells)
    b = np.zeros((3, p.cells))
    sums = np.zeros((p.batch, 5))
    lib().ora_moments(dims.ctypes.data_as(_ip), float(p.c_l), float(p.kappa),
                      solid.ctypes.data_as(_u8p) if solid is not None else None,
                      _d(S), _d(n), _d(e), _d(b), _d(sums))
    return n, e, b, sums


def adjoint_step(p: Problem, Sg, lam_next, per_cell: bool = False):
    """One g-only reverse step; returns (lam_t, dL/dtau[batch], dL/dbeta_in[3], dL/de_in)
    and, with per_cell, also dL/dtau(x)[cells] (the per-cell relaxation times)."""
    if p.eta_s > 0:
        raise ValueError("the g-only reverse step does not hold while eta/s is held")
    args, rx = p._args()
    Sg, lam_next = _f64(Sg), _f64(lam_next)
    lam_out = np.zeros((Q, p.cells))
    dtau = np.zeros(p.batch)
    dbin = np.zeros(3)
    dein = np.zeros(1)
    dcell = np.zeros(p.cells)
    lib().ora_adjoint_step(*args, rx, _d(Sg), _d(lam_next), _d(lam_out), _d(dtau),
                           _d(dbin), _d(dein), _d(dcell))
    if per_cell:
        return lam_out, dtau, dbin, dein[0], dcell
    return lam_out, dtau, dbin, dein[0]


def moments_adjoint(p: Problem, Sg, dLde, dLdb):
    dims = np.array([p.nx, p.ny, p.nz, p.batch], dtype=np.int32)
    solid = None if p.solid is None else np.ascontiguousarray(p.solid.reshape(-1).astype(np.uint8))
    Sg, dLde, dLdb = _f64(Sg), _f64(dLde).reshape(-1), _f64(dLdb).reshape(3, -1)
    lam = np.zeros((Q, p.cells))
    lib().ora_moments_adjoint(dims.ctypes.data_as(_ip), float(p.c_l), float(p.kappa),
                              solid.ctypes.data_as(_u8p) if solid is not None else None,
                              _d(Sg), _d(dLde), _d(np.ascontiguousarray(dLdb)), _d(lam))
    return lam


def init_adjoint(p: Problem, e0, beta0, lam0):
    args, _ = p._args()
    e0, beta0, lam0 = _f64(e0).reshape(-1), _f64(beta0).reshape(3, -1), _f64(lam0)
    de0 = np.zeros(p.cells)
    db0 = np.zeros((3, p.cells))
    dbin = np.zeros(3)
    dein = np.zeros(1)
    lib().ora_init_adjoint(*args, float(p.kappa), _d(e0), _d(np.ascontiguousarray(beta0)),
                           _d(lam0), _d(de0),
                           _d(db0), _d(dbin), _d(dein))
    return de0, db0, dbin, dein[0]


@dataclass
class Loss:
    """L = sum a (e - t)^2 + sum be*e + sum bb.beta over non-solid cells."""

    a: Optional[np.ndarray] = None
    t: Optional[np.ndarray] = None
    be: Optional[np.ndarray] = None
    bb: Optional[np.ndarray] = None  # [3][cells]

    def ptrs(self):
        self._keep = [_f64(v).reshape(-1) if v is not None else None
                      for v in (self.a, self.t, self.be, self.bb)]
        return [_d(v) if v is not None else None for v in self._keep]


def loss(p: Problem, e0, beta0, nsteps, L: Loss) -> float:
    if p.eta_s > 0:
        raise ValueError("g-only runs do not hold eta/s")
    args, rx = p._args()
    e0, beta0 = _f64(e0).reshape(-1), np.ascontiguousarray(_f64(beta0).reshape(3, -1))
    return float(lib().ora_loss(*args, rx, _d(e0), _d(beta0), int(nsteps), *L.ptrs()))


def loss_cs(p: Problem, e0, beta0, nsteps, L: Loss, d_tau=None, d_inflow=None, d_e0=None,
            d_beta0=None, d_tau_cell=None):
    """Complex-step directional derivative dL.d; returns (L, dL.d).  d_tau_cell
    perturbs the per-cell relaxation times (needs p.tau_cell)."""
    if p.eta_s > 0:
        raise ValueError("g-only runs do not hold eta/s")
    assert d_tau_cell is None or p.tau_cell is not None
    args, rx = p._args()
    e0, beta0 = _f64(e0).reshape(-1), np.ascontiguousarray(_f64(beta0).reshape(3, -1))
    dt, di, de, db, dc = (_f64(v).reshape(-1) if v is not None else None
                          for v in (d_tau, d_inflow, d_e0, d_beta0, d_tau_cell))
    lv = np.zeros(1)
    r = lib().ora_loss_cs(*args, rx, _d(e0), _d(beta0), int(nsteps), *L.ptrs(),
                          _d(dt), _d(di), _d(de), _d(db), _d(dc), _d(lv))
    return float(lv[0]), float(r)


@dataclass
class Gradient:
    loss: float
    tau: np.ndarray
    e_in: float
    beta_in: np.ndarray
    e0: np.ndarray
    beta0: np.ndarray
    tau_cell: np.ndarray  # dL/dtau(x): the gradient with respect to per-cell relaxation times


def gradient(p: Problem, e0, beta0, nsteps, L: Loss) -> Gradient:
    """Store-all FP64 reverse sweep of a g-only run (oracle's own adjoint)."""
    if p.eta_s > 0:
        raise ValueError("g-only runs do not hold eta/s")
    args, rx = p._args()
    e0, beta0 = _f64(e0).reshape(-1), np.ascontiguousarray(_f64(beta0).reshape(3, -1))
    gt = np.zeros(p.batch)
    gi = np.zeros(4)
    ge = np.zeros(p.cells)
    gb = np.zeros((3, p.cells))
    gc = np.zeros(p.cells)
    lv = lib().ora_gradient(*args, rx, _d(e0), _d(beta0), int(nsteps), *L.ptrs(),
                            _d(gt), _d(gi), _d(ge), _d(gb), _d(gc))
    return Gradient(float(lv), gt, float(gi[0]), gi[1:4].copy(), ge, gb, gc)


def transport(p: Problem, S: np.ndarray):
    """(T, s, eta, eta/s) per cell of a stored f+g state ([2][19][cells]), each
    cell with its relaxation time (per instance, per-cell field, or the eta/s
    rule at its fields); zeros on solid cells."""
    dims = np.array([p.nx, p.ny, p.nz, p.batch], dtype=np.int32)
    _, rx = p._args()
    solid = None if p.solid is None else np.ascontiguousarray(p.solid.reshape(-1).astype(np.uint8))
    out = [np.zeros(p.cells) for _ in range(4)]
    ok = lib().ora_transport(dims.ctypes.data_as(_ip), float(p.c_l),
                             solid.ctypes.data_as(_u8p) if solid is not None else None, _d(S),
                             rx, *[_d(o) for o in out])
    if not ok:
        raise ValueError("transport quantities are defined for e = 3P matter (kappa = 1/3)")
    return tuple(out)
