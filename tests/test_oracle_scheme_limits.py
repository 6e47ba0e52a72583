"""Where the scheme itself (as published, c_l = 1) stops being valid.

These behaviours are properties of the method, shown on the oracle, not of any
kernel; the GPU path reproduces them and the workloads account for them.
"""
import numpy as np

import oracle
import rlb_inputs as ri
from helpers import problem
from oracle import d1q3


def test_reduced_sphere_setup_goes_unphysical_after_the_shock_meets_the_sphere():
    """The obstacle set-up (|beta_in| = 0.5, e_in/e = 5, tau = 0.55) at a quarter of
    its size: physical while the shock approaches, unphysical (|M| > E) within a
    few steps of reaching the sphere."""
    s = ri.sphere(nx=50, ny=26, nz=26, centre=(15, 13, 13), radius=4)
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    assert oracle.run(p, S, 10) == 0
    bad = oracle.run(p, S, 30)
    assert bad > 0


def test_transverse_asymmetry_grows_on_a_strong_shock_tube():
    """1 x 1 x 800 tube at e_L/e_R = 16: the oracle's own trajectory keeps the
    mirror symmetry of the 1-D flow, but a 1e-15 relative asymmetry between the
    (+x,+z) and (-x,+z) populations grows by orders of magnitude while a
    longitudinal perturbation of the same size does not."""
    s = ri.shock_tube()
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    St = S.copy()
    St[1, 11] *= 1 + 1e-15
    St[1, 14] *= 1 - 1e-15
    Sl = S.copy()
    Sl[1, 5] *= 1 + 1e-15
    for A in (S, St, Sl):
        oracle.run(p, A, 100)
    scale = np.abs(S[1]).max()
    d_t = np.abs(St[1] - S[1]).max() / scale
    d_l = np.abs(Sl[1] - S[1]).max() / scale
    assert d_t > 1e-7
    assert d_l < 1e-13


def test_one_dimensional_tube_fails_above_pressure_ratio_about_19():
    """Lumped 1-D form (exact for tubes): e_L/e_R = 27 goes unphysical within 200
    steps, e_L/e_R = 15 stays physical for 2000 steps (tau = 0.66, 2048 cells)."""
    z = np.arange(2048)
    for ratio, steps, ok in ((27.0, 200, False), (15.0, 2000, True)):
        e0 = np.where(z < 1024, 1.0, 1.0 / ratio)
        with np.errstate(all="ignore"):
            n, e, b = d1q3.run(e0 ** 0.75, e0, np.zeros(2048), 0.66, 1.0, steps)
        phys = np.isfinite(e).all() and (e > 0).all() and (np.abs(b) < 1).all()
        assert phys == ok, (ratio, phys)
