"""Pins of the oracle's derivatives.

Three independent routes to the same numbers must agree:
  * central finite differences of the plain FP64 forward run (real arithmetic);
  * complex-step differentiation of the whole run (exact to rounding);
  * the oracle's store-all reverse sweep (transpose of the pull map, built from
    per-cell complex-step collision Jacobians).
"""
import numpy as np
import pytest

import oracle
import rlb_inputs as ri
from test_oracle_pins import problem


def tube(batch=2, nz=48, steps=40):
    s = ri.shock_tube(nz=nz, e_L=1.0, e_R=0.3, tau=0.7, steps=steps, batch=batch)
    s.tau = np.array([0.7, 0.85][:batch])
    return s


def sphere_small(steps=12):
    s = ri.random_state_setup(
        10, 6, 7, seed=21, tau=[0.75],
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
        inflow=(1.0, 1.0, 0.2, 0.03, 0.0), solid_centre=(5, 3, 3), solid_radius=1.5)
    s.steps = steps
    return s


def loss_for(s, seed=0):
    rng = np.random.default_rng(seed)
    C = s.cells
    return oracle.Loss(a=rng.uniform(0.5, 1.5, C), t=rng.uniform(0.2, 1.0, C),
                       be=rng.standard_normal(C) * 0.1, bb=rng.standard_normal((3, C)) * 0.1)


@pytest.mark.parametrize("make", [tube, sphere_small])
def test_complex_step_matches_central_fd(make):
    s = make()
    p = problem(s)
    L = loss_for(s)
    rng = np.random.default_rng(1)
    d_tau = rng.standard_normal(s.batch)
    d_e0 = rng.standard_normal(s.cells) * 0.05
    d_in = np.array([0.1, 0.3, -0.2, 0.1])
    L0, dcs = oracle.loss_cs(p, s.e0, s.beta0, s.steps, L, d_tau=d_tau, d_e0=d_e0, d_inflow=d_in)
    assert L0 == pytest.approx(oracle.loss(p, s.e0, s.beta0, s.steps, L), rel=1e-14)
    # FD rounding noise is ~ 1e-16 |L| / h, truncation ~ h^2: h = 1e-5 balances them
    h = 1e-5

    def shifted(sign):
        s2 = s.with_(tau=s.tau + sign * h * d_tau, e0=s.e0 + sign * h * d_e0,
                     inflow=tuple(np.array(s.inflow) + sign * h * np.concatenate([[0.0], d_in])))
        return oracle.loss(problem(s2), s2.e0, s2.beta0, s.steps, L)

    fd = (shifted(+1) - shifted(-1)) / (2 * h)
    assert fd == pytest.approx(dcs, rel=1e-6, abs=1e-10 * abs(L0))


@pytest.mark.parametrize("make", [tube, sphere_small])
def test_store_all_reverse_matches_complex_step(make):
    """Adjoint dot-product identity: <grad, d> from the reverse sweep equals the
    complex-step directional derivative, for several random directions."""
    s = make()
    p = problem(s)
    L = loss_for(s, seed=3)
    G = oracle.gradient(p, s.e0, s.beta0, s.steps, L)
    rng = np.random.default_rng(2)
    for k in range(3):
        d_tau = rng.standard_normal(s.batch)
        d_e0 = rng.standard_normal(s.cells)
        d_b0 = rng.standard_normal((3, s.cells)) * 0.3
        d_in = rng.standard_normal(4)
        _, dcs = oracle.loss_cs(p, s.e0, s.beta0, s.steps, L, d_tau=d_tau, d_e0=d_e0,
                                d_beta0=d_b0, d_inflow=d_in)
        adj = (G.tau @ d_tau + G.e0 @ d_e0 + (G.beta0 * d_b0).sum()
               + G.e_in * d_in[0] + G.beta_in @ d_in[1:])
        assert adj == pytest.approx(dcs, rel=1e-11, abs=1e-13 * abs(G.loss))


def test_adjoint_step_is_transpose_of_step():
    """Per step: <lam, J v> = <J^T lam, v>, with J v by central differences of the
    plain FP64 step (g population, outflow + inflow + bounce-back lattice)."""
    s = sphere_small()
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, 3)
    Sg = np.ascontiguousarray(S[1])
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(Sg.shape)
    v = rng.standard_normal(Sg.shape) * np.abs(Sg).mean()
    solid = s.solid.astype(bool)
    v[:, solid] = 0.0
    lam_t, _, _, _ = oracle.adjoint_step(p, Sg, lam)
    h = 1e-6

    def stepped(x):
        x = np.ascontiguousarray(x.copy())
        oracle.run_g(p, x, 1)
        return x

    Jv = (stepped(Sg + h * v) - stepped(Sg - h * v)) / (2 * h)
    lhs = (lam * Jv).sum()
    rhs = (lam_t * v).sum()
    assert lhs == pytest.approx(rhs, rel=1e-7)
