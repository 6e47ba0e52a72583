"""Seeded synthetic problem set-ups shared by the oracle and the GPU path.

This module only describes problems: extents, boundary codes, relaxation times,
initial (n, e, beta) fields and solid masks, all drawn from numpy's PCG64 with
fixed seeds in FP64.  It holds none of the scheme's arithmetic (no equilibria,
moments, streaming or collision), and neither the oracle nor the GPU library is
imported here.

Workloads follow the paper's set-ups (shock-tube section; Fig. 1's sphere run)
with sizes and values fixed by this project:

  * ``shock_tube``: 1 x 1 x 800, e = 1 on the left half, 1/16 on the right,
    beta = 0, n = e^(3/4) (n ~ T^3 with e ~ T^4), tau = 0.6, outflow in z.
  * ``tachyon_tube``: the same tube at lattice speed c_l = 10, tau = 0.51,
    4000 steps (time 400).
  * ``sphere``: 200 x 100 x 100, solid ball of radius 15 at (60, 50, 50),
    inflow plane x = 0 at (n, e, beta) = (1, 1, (0.5, 0, 0)), downstream e = 0.2 at
    rest, tau = 0.55, outflow at x = nx-1, y and z periodic.
  * ``periodic_box``: 256^3 periodic, smooth random beta from 8 Fourier modes
    (|beta| <= 0.2) and e = 1 + 0.1 s(x).
  * ``tube_batch``: 64 tubes of 1 x 1 x 2048 with tau_b ~ U[0.51, 1] and
    e_L/e_R ~ U[4, 32].
  * ``sphere_large``: 384 x 192 x 192 with a radius-24 sphere at (115, 96, 96);
    ``sphere_large_steady``: the same with |beta_in| = 0.3 into e = 1 at rest.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

PERIODIC, OUTFLOW, INFLOW = 0, 1, 2

# Storage and collision-type codes (same numbering as the C header's enums).
F64, F32, F32DEV, F16DEV, BF16DEV = 0, 1, 2, 3, 4
COLLIDE_AUTO, COLLIDE_F32, COLLIDE_F64, COLLIDE_F32_MOM64 = 0, 1, 2, 3
STORAGE_NAMES = {F64: "f64", F32: "f32", F32DEV: "f32dev", F16DEV: "f16dev", BF16DEV: "bf16dev"}


@dataclass
class Setup:
    """One problem: geometry, boundaries, parameters and initial fields."""

    name: str
    nx: int
    ny: int
    nz: int
    batch: int = 1
    c_l: float = 1.0
    bc: Tuple[Tuple[int, int], ...] = ((PERIODIC, PERIODIC),) * 3
    inflow: Tuple[float, ...] = (1.0, 1.0, 0.0, 0.0, 0.0)  # n, e, beta_x, beta_y, beta_z
    tau: np.ndarray = field(default_factory=lambda: np.array([0.6]))
    steps: int = 100
    storage: int = F64
    collide: int = COLLIDE_AUTO
    n_ref: float = 1.0
    e_ref: float = 1.0
    n0: Optional[np.ndarray] = None  # [cells]
    e0: Optional[np.ndarray] = None  # [cells]
    beta0: Optional[np.ndarray] = None  # [3][cells]
    solid: Optional[np.ndarray] = None  # uint8 [cells]
    tau_cell: Optional[np.ndarray] = None  # [cells]: per-cell relaxation times (else tau)
    eta_s: float = 0.0  # > 0: hold eta/s fixed (tau from the local state)
    d_G: float = 16.0  # degeneracy in n_eq = d_G T^3 / pi^2
    kappa: float = 1.0 / 3.0  # equation of state P = kappa e
    inplace: bool = False  # one state buffer, in-place (AA-pattern) streaming

    @property
    def cells(self) -> int:
        return self.batch * self.nz * self.ny * self.nx

    def coords(self):
        """Integer cell coordinates (b, z, y, x) broadcastable to [batch, nz, ny, nx]."""
        b = np.arange(self.batch).reshape(-1, 1, 1, 1)
        z = np.arange(self.nz).reshape(1, -1, 1, 1)
        y = np.arange(self.ny).reshape(1, 1, -1, 1)
        x = np.arange(self.nx).reshape(1, 1, 1, -1)
        return b, z, y, x

    def with_(self, **kw) -> "Setup":
        return replace(self, **kw)


def _fields(s: Setup, e, beta, n=None):
    shape = (s.batch, s.nz, s.ny, s.nx)
    e = np.broadcast_to(np.asarray(e, dtype=np.float64), shape).reshape(-1).copy()
    if n is None:
        n = e ** 0.75
    else:
        n = np.broadcast_to(np.asarray(n, dtype=np.float64), shape).reshape(-1).copy()
    beta = np.stack([np.broadcast_to(np.asarray(bk, dtype=np.float64), shape).reshape(-1)
                     for bk in beta]).copy()
    return n, e, beta


def ball(s: Setup, centre, radius) -> np.ndarray:
    """uint8 mask: 1 where (x-cx)^2 + (y-cy)^2 + (z-cz)^2 <= r^2 on integer indices."""
    b, z, y, x = s.coords()
    cx, cy, cz = centre
    m = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= radius ** 2
    return np.broadcast_to(m, (s.batch, s.nz, s.ny, s.nx)).reshape(-1).astype(np.uint8)


def shock_tube(nz=800, e_L=1.0, e_R=1.0 / 16.0, tau=0.6, steps=500, c_l=1.0, batch=1,
               storage=F64) -> Setup:
    """Riemann problem along z: cells k < nz/2 hold e_L, the rest e_R, beta = 0."""
    s = Setup("shock_tube", 1, 1, nz, batch=batch, c_l=c_l,
              bc=((PERIODIC, PERIODIC), (PERIODIC, PERIODIC), (OUTFLOW, OUTFLOW)),
              tau=np.full(batch, float(tau)), steps=steps, storage=storage)
    b, z, y, x = s.coords()
    e_L = np.asarray(e_L, dtype=np.float64).reshape(-1, 1, 1, 1)
    e_R = np.asarray(e_R, dtype=np.float64).reshape(-1, 1, 1, 1)
    e = np.where(z < nz // 2, e_L, e_R)
    s.n0, s.e0, s.beta0 = _fields(s, e, (0.0, 0.0, 0.0))
    return s


def tachyon_tube(nz=800, t=400, c_l=10.0, tau=0.51, ratio=16.0, storage=F64) -> Setup:
    """The shock-tube section's "numerical tachyons": the ratio-16 tube (star
    state beta* = 0.54, above the c_l = 1 positivity bound c_l/3) run with a
    lattice speed c_l = 10, up to time t (in cells / c: t * c_l steps).  tau =
    0.51 gives the kinematic viscosity c_l (tau - 1/2) / 3 = 0.033 of the c_l = 1
    tube at tau = 0.6."""
    s = shock_tube(nz=nz, e_L=1.0, e_R=1.0 / ratio, tau=tau, steps=int(round(t * c_l)),
                   c_l=c_l, storage=storage)
    s.name = "tachyon_tube"
    return s


def sphere(nx=200, ny=100, nz=100, centre=(60, 50, 50), radius=15, beta_in=0.5, e_in=1.0,
           e_down=0.2, tau=0.55, steps=2000, storage=F64, c_l=1.0) -> Setup:
    """Relativistic shock on a fixed sphere (Fig. 1's set-up, sizes fixed here)."""
    s = Setup("sphere", nx, ny, nz, c_l=c_l,
              bc=((INFLOW, OUTFLOW), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)),
              inflow=(e_in ** 0.75, e_in, beta_in, 0.0, 0.0),
              tau=np.array([float(tau)]), steps=steps, storage=storage)
    s.solid = ball(s, centre, radius)
    s.n0, s.e0, s.beta0 = _fields(s, e_down, (0.0, 0.0, 0.0))
    return s


def _fourier(rng, shape_zyx, nmodes, vector, kmax=4):
    nz, ny, nx = shape_zyx
    z = np.arange(nz).reshape(-1, 1, 1)
    y = np.arange(ny).reshape(1, -1, 1)
    x = np.arange(nx).reshape(1, 1, -1)
    comps = 3 if vector else 1
    out = np.zeros((comps, nz, ny, nx))
    for _ in range(nmodes):
        while True:
            m = rng.integers(-kmax, kmax + 1, size=3)
            if np.any(m != 0):
                break
        a = rng.standard_normal(comps)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        arg = 2 * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz) + ph
        s = np.sin(arg)
        for c in range(comps):
            out[c] += a[c] * s
    return out


def periodic_box(n=256, steps=1000, storage=F64, beta_max=0.2, de=0.1, tau=0.6, c_l=1.0,
                 nx=None, ny=None, nz=None, seed_beta=0, seed_e=1) -> Setup:
    """Periodic box with smooth random fields: beta = sum of 8 Fourier modes scaled
    to max |beta| = beta_max, e = 1 + de * s(x) with s a scalar 8-mode field scaled
    to max |s| = 1, n = e^(3/4)."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    s = Setup("periodic_box", nx, ny, nz, c_l=c_l, tau=np.array([float(tau)]), steps=steps,
              storage=storage)
    bv = _fourier(np.random.default_rng(seed_beta), (nz, ny, nx), 8, True)
    bv *= beta_max / np.sqrt((bv ** 2).sum(axis=0)).max()
    sv = _fourier(np.random.default_rng(seed_e), (nz, ny, nx), 8, False)[0]
    sv /= np.abs(sv).max()
    e = 1.0 + de * sv
    s.n0, s.e0, s.beta0 = _fields(s, e[None], (bv[0][None], bv[1][None], bv[2][None]))
    return s


def tube_batch(batch=64, nz=2048, steps=2000, storage=F32, seed=2, tau_range=(0.51, 1.0),
               ratio_range=(4.0, 32.0), reject=None):
    """Batch of independent shock tubes with tau_b ~ U[tau_range] and
    e_L/e_R = r_b ~ U[ratio_range] (e_L = 1).

    ``reject`` (optional) is a callable taking (tau, ratio) arrays and returning
    the indices of instances to draw again (for instance those a screening run
    found unphysical); they are redrawn from the same seeded stream, in index
    order, until none is rejected.  Returns (setup, tau, ratio, n_redrawn)."""
    rng = np.random.default_rng(seed)
    tau = rng.uniform(*tau_range, size=batch)
    ratio = rng.uniform(*ratio_range, size=batch)
    redrawn = 0
    while reject is not None:
        bad = sorted(int(i) for i in reject(tau.copy(), ratio.copy()))
        if not bad:
            break
        for i in bad:
            tau[i] = rng.uniform(*tau_range)
            ratio[i] = rng.uniform(*ratio_range)
            redrawn += 1
    s = shock_tube(nz=nz, e_L=np.ones(batch), e_R=1.0 / ratio, tau=0.6, steps=steps,
                   batch=batch, storage=storage)
    s.name = "tube_batch"
    s.tau = tau.copy()
    return s, tau, ratio, redrawn


def sphere_large(steps=4000, storage=F32, beta_in=0.5, e_down=0.2) -> Setup:
    s = sphere(nx=384, ny=192, nz=192, centre=(115, 96, 96), radius=24, steps=steps,
               storage=storage, beta_in=beta_in, e_down=e_down)
    s.name = "sphere_large"
    return s


def sphere_large_steady(steps=4000, storage=F32) -> Setup:
    """The 384 x 192 x 192 sphere with a milder inflow that stays physical at
    c_l = 1 for the 4000 steps: |beta_in| = 0.3 into fluid at rest at the
    inflow's own energy density (e_down = 1), so no pressure jump travels."""
    s = sphere_large(steps=steps, storage=storage, beta_in=0.3, e_down=1.0)
    s.name = "sphere_large_steady"
    return s


def random_state_setup(nx, ny, nz, batch=1, bc=((PERIODIC, PERIODIC),) * 3, c_l=1.0,
                       seed=7, beta_max=0.15, de=0.2, tau=None, solid_centre=None,
                       solid_radius=None, inflow=(1.0, 1.0, 0.0, 0.0, 0.0),
                       storage=F64) -> Setup:
    """Small lattice with smooth random fields for parity tests (any boundaries)."""
    rng = np.random.default_rng(seed)
    if tau is None:
        tau = rng.uniform(0.55, 1.2, size=batch)
    s = Setup("random", nx, ny, nz, batch=batch, c_l=c_l, bc=bc, inflow=tuple(inflow),
              tau=np.asarray(tau, dtype=np.float64).reshape(-1), steps=10, storage=storage)
    shape = (nz, ny, nx)
    bv = np.stack([_fourier(rng, shape, 6, True, kmax=2) for _ in range(batch)], axis=1)
    bv *= beta_max / max(np.sqrt((bv ** 2).sum(axis=0)).max(), 1e-30)
    sv = np.stack([_fourier(rng, shape, 6, False, kmax=2)[0] for _ in range(batch)])
    sv /= max(np.abs(sv).max(), 1e-30)
    e = 1.0 + de * sv
    s.n0, s.e0, s.beta0 = _fields(s, e, (bv[0], bv[1], bv[2]))
    if solid_centre is not None:
        s.solid = ball(s, solid_centre, solid_radius)
    return s
