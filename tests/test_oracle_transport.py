"""Pins of the oracle's transport quantities, per-cell relaxation times and
eta/s-holding rule (the viscosity relation at the end of the equilibrium
section, and the temperature, equilibrium density, fugacity and entropy
density of the shock-tube section).

Each quantity is checked against something other than its own formula: the
closed forms of the entropy at fixed fugacity, the decay rate of a shear wave
measured from the scheme's dynamics, bitwise identities between the per-cell
and per-instance relaxation paths, and complex-step derivatives against the
reverse sweep.
"""
import math

import numpy as np
import pytest

import oracle
import rlb_inputs as ri
from test_oracle_pins import golden


def uniform_state(p, n, e, beta=(0.0, 0.0, 0.0)):
    C = p.cells
    b = np.zeros((3, C))
    for k in range(3):
        b[k] = beta[k]
    return oracle.init(p, np.full(C, n), np.full(C, e), b)


@pytest.mark.parametrize("log_lambda", [0.0, 1.0, -0.7])
def test_entropy_per_particle_is_four_minus_log_fugacity(log_lambda):
    """At temperature T (from e = 3 n T) the equilibrium density is
    n_eq = d_G T^3 / pi^2 (d_G = 16 for gluons, T0 of the paper's tube); a gas
    with n = exp(log_lambda) n_eq has s / n = 4 - log_lambda, so the
    equilibrated gas (lambda = 1) has s = 4 n."""
    g = golden()
    d_G, T0 = g["d_G_gluons"], g["T0_lattice"]
    n = math.exp(log_lambda) * d_G * T0 ** 3 / math.pi ** 2
    e = 3.0 * n * T0
    p = oracle.Problem(3, 2, 2, tau=(0.7,), d_G=d_G)
    S = uniform_state(p, n, e)
    T, s, eta, eos = oracle.transport(p, S)
    assert np.allclose(T, T0, rtol=1e-13)
    assert np.allclose(s / n, 4.0 - log_lambda, rtol=1e-12)


def _shear_decay(p, L, steps0=200, steps=800, amp=1e-4):
    """Measured per-step decay rate of beta_y = amp sin(2 pi z / L) on a
    1 x 1 x L periodic tube, and the transport quantities of the start state."""
    z = np.arange(L)
    C = p.cells
    b = np.zeros((3, C))
    b[1] = amp * np.sin(2 * np.pi * z / L)
    S = oracle.init(p, np.ones(C), np.ones(C), b)
    tr = oracle.transport(p, S)
    mode = np.sin(2 * np.pi * z / L)
    oracle.run(p, S, steps0)
    a1 = oracle.moments(p, S)[2][1] @ mode
    oracle.run(p, S, steps)
    a2 = oracle.moments(p, S)[2][1] @ mode
    return -math.log(a2 / a1) / steps, tr


@pytest.mark.parametrize("tau,c_l", [(0.8, 1.0), (0.65, 2.0)])
def test_viscosity_matches_the_measured_shear_wave_decay(tau, c_l):
    """The kinematic viscosity nu = eta / ((e + P) gamma^2) built from the
    oracle's eta sets the decay of a shear wave: amplitude ~ exp(-nu k^2 t),
    t = steps * dt with dt = dx / c_l."""
    L = 128
    p = oracle.Problem(1, 1, L, c_l=c_l, tau=(tau,))
    rate, (T, s, eta, eos) = _shear_decay(p, L)
    nu = eta.mean() / (4.0 / 3.0 * 1.0)  # e = 1, gamma = 1 to O(amp^2)
    want = nu * (2 * np.pi / L) ** 2 / c_l
    assert rate == pytest.approx(want, rel=2e-3)


def test_uniform_tau_field_equals_per_instance_tau_bitwise():
    """A per-cell field holding each instance's tau reproduces the
    per-instance run exactly (two instances, different tau)."""
    s = ri.random_state_setup(5, 4, 6, batch=2, seed=31, tau=[0.62, 0.95],
                              bc=((ri.OUTFLOW, ri.OUTFLOW), (0, 0), (0, 0)))
    p = oracle.Problem(s.nx, s.ny, s.nz, s.batch, s.c_l, s.bc, s.inflow, s.tau, s.solid)
    per = s.nx * s.ny * s.nz
    pc = oracle.Problem(s.nx, s.ny, s.nz, s.batch, s.c_l, s.bc, s.inflow, (7.0, 7.0), s.solid,
                        tau_cell=np.repeat(np.asarray(s.tau, float), per))
    A = oracle.init(p, s.n0, s.e0, s.beta0)
    B = A.copy()
    oracle.run(p, A, 15)
    oracle.run(pc, B, 15)
    assert np.array_equal(A, B)


def test_tau_field_acts_per_cell():
    """Every cell of a periodic row holds the same (non-equilibrium)
    populations, so streaming leaves them in place and one step is one
    collision per cell: cells with tau = 0.6 and tau = 1.4 must come out as
    single-cell collisions with their own tau."""
    p0 = oracle.Problem(4, 1, 1, tau=(0.7,))
    S = uniform_state(p0, 1.0, 1.0)
    rng = np.random.default_rng(3)
    S = np.ascontiguousarray(S + 1e-3 * rng.standard_normal((2, 19, 1)))
    tc = np.array([0.6, 0.6, 1.4, 1.4])
    p = oracle.Problem(4, 1, 1, tau=(0.7,), tau_cell=tc)
    S1 = S.copy()
    oracle.run(p, S1, 1)
    for x in range(4):
        of, og, _ = oracle.collide(S[0, :, x], S[1, :, x], tc[x], 1.0)
        assert np.array_equal(S1[0, :, x], of) and np.array_equal(S1[1, :, x], og)
    assert np.abs(S1[1, :, 0] - S1[1, :, 2]).max() > 1e-6  # the two taus differ


def test_holding_eta_over_s_sets_the_decay_rate():
    """With eta/s held fixed the relaxation time comes from the local state;
    on a near-uniform state the shear wave then decays with
    nu = (eta/s) s / ((e + P) gamma^2), and the diagnostics report eta/s."""
    L = 128
    eta_s = 0.08
    p = oracle.Problem(1, 1, L, tau=(0.7,), eta_s=eta_s, d_G=16.0)
    rate, (T, s, eta, eos) = _shear_decay(p, L)
    assert np.allclose(eos, eta_s, rtol=1e-12)
    nu = eta_s * s.mean() / (4.0 / 3.0)
    want = nu * (2 * np.pi / L) ** 2
    assert rate == pytest.approx(want, rel=2e-3)
    # the same run with the per-cell tau that the rule gives is identical to
    # first order: the uniform tau from the start state reproduces the rate
    tau_rule = 0.5 + 9.0 * eta_s * s.mean() / (4.0 * 1.0)
    rate2, _ = _shear_decay(oracle.Problem(1, 1, L, tau=(tau_rule,)), L)
    assert rate == pytest.approx(rate2, rel=1e-6)


def test_tau_cell_gradient_matches_complex_step_and_sums_to_instance_gradient():
    s = ri.random_state_setup(6, 5, 7, batch=2, seed=32, tau=[0.7, 0.9],
                              bc=((ri.INFLOW, ri.OUTFLOW), (0, 0), (ri.OUTFLOW, ri.OUTFLOW)),
                              inflow=(1.0, 1.1, 0.1, 0.0, 0.02), solid_centre=(3, 2, 3),
                              solid_radius=1.5)
    rng = np.random.default_rng(5)
    C = s.cells
    tc = rng.uniform(0.6, 1.0, C)
    p = oracle.Problem(s.nx, s.ny, s.nz, s.batch, s.c_l, s.bc, s.inflow, s.tau, s.solid,
                       tau_cell=tc)
    Lo = oracle.Loss(a=rng.uniform(0.5, 1.5, C), t=rng.uniform(0.2, 1.0, C),
                     bb=rng.standard_normal((3, C)) * 0.1)
    steps = 12
    G = oracle.gradient(p, s.e0, s.beta0, steps, Lo)
    v = rng.standard_normal(C)
    _, cs = oracle.loss_cs(p, s.e0, s.beta0, steps, Lo, d_tau_cell=v)
    assert G.tau_cell @ v == pytest.approx(cs, rel=1e-9)
    per = s.nx * s.ny * s.nz
    for b in range(s.batch):
        assert G.tau_cell[b * per:(b + 1) * per].sum() == pytest.approx(G.tau[b], rel=1e-12)
        ones = np.zeros(C)
        ones[b * per:(b + 1) * per] = 1.0
        _, csb = oracle.loss_cs(p, s.e0, s.beta0, steps, Lo, d_tau_cell=ones)
        assert G.tau[b] == pytest.approx(csb, rel=1e-9)
    # solid cells carry no gradient
    assert np.all(G.tau_cell[s.solid.reshape(-1) != 0] == 0.0)
