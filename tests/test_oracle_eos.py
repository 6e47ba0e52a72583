"""Pins of the oracle's general equation of state P = kappa e (eqs. equil1,
equil2a, equil2b and the inversion of the macroscopic constraints for that
EoS).

Checked against the relativistic moments the equilibria must reproduce
(N^mu and T^{mu nu} = P eta^{mu nu} + (e+P) u^mu u^nu with P = kappa e), the
inversion round trip, the ultra-relativistic forms at kappa -> 1/3, the sound
speed sqrt(kappa) of the resulting fluid, and the reverse sweep against
complex-step derivatives.
"""
import math

import numpy as np
import pytest

import oracle
import rlb_inputs as ri
from helpers import problem


@pytest.mark.parametrize("kappa", [0.15, 0.25, 0.5, 0.9])
@pytest.mark.parametrize("c_l", [1.0, 2.0])
def test_general_equilibrium_moments_equal_relativistic_moments(kappa, c_l):
    rng = np.random.default_rng(21)
    e, w, _ = oracle.lattice()
    c = c_l * e
    for _ in range(30):
        v = rng.standard_normal(3)
        beta = v / np.linalg.norm(v) * rng.uniform(0.0, 0.9)
        n, eps = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0)
        feq, geq = oracle.equilibria(n, eps, beta, c_l, kappa)
        g2 = 1.0 / (1.0 - beta @ beta)
        P = kappa * eps
        W = (eps + P) * g2
        assert abs(feq.sum() - n * math.sqrt(g2)) <= 1e-14 * n * math.sqrt(g2)
        assert np.abs(feq @ c - n * math.sqrt(g2) * beta).max() <= 1e-14 * n * math.sqrt(g2) * c_l
        assert abs(geq.sum() - (W - P)) <= 1e-14 * W
        assert np.abs(geq @ c - W * beta).max() <= 1e-14 * W * c_l
        T_ij = np.einsum("q,qa,qb->ab", geq, c, c)
        assert np.abs(T_ij - (P * np.eye(3) + W * np.outer(beta, beta))).max() <= 1e-14 * W * c_l ** 2


@pytest.mark.parametrize("kappa", [0.1, 0.25, 0.6, 1.0])
def test_general_inversion_round_trip(kappa):
    rng = np.random.default_rng(22)
    e, _, _ = oracle.lattice()
    for c_l in (1.0, 2.0):
        for _ in range(30):
            v = rng.standard_normal(3)
            beta = v / np.linalg.norm(v) * rng.uniform(0.0, 0.9)
            n, eps = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0)
            feq, geq = oracle.equilibria(n, eps, beta, c_l, kappa)
            nn, ee, bb, ok = oracle.invert(feq.sum(), geq.sum(), geq @ (c_l * e), kappa)
            assert ok
            assert nn == pytest.approx(n, rel=1e-13)
            assert ee == pytest.approx(eps, rel=1e-13)
            assert np.abs(bb - beta).max() <= 1e-13


def test_general_forms_reduce_to_the_ultra_relativistic_ones():
    """At kappa = 1/3 (approached from above, which takes the general branch)
    eqs. equil2a/equil2b equal equil2as/equil2bs and the general inversion the
    e = 3P one."""
    rng = np.random.default_rng(23)
    k = 1.0 / 3.0 + 1e-15
    e, _, _ = oracle.lattice()
    for c_l in (1.0, 2.0, 10.0):
        for _ in range(20):
            v = rng.standard_normal(3)
            beta = v / np.linalg.norm(v) * rng.uniform(0.0, 0.9)
            n, eps = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0)
            f1, g1 = oracle.equilibria(n, eps, beta, c_l)
            f2, g2 = oracle.equilibria(n, eps, beta, c_l, k)
            assert np.abs(g2 - g1).max() <= 1e-13 * np.abs(g1).max()
            assert np.abs(f2 - f1).max() <= 1e-15 * np.abs(f1).max()
            m = g1 @ (c_l * e)
            a = oracle.invert(f1.sum(), g1.sum(), m)
            b = oracle.invert(f1.sum(), g1.sum(), m, k)
            assert b[1] == pytest.approx(a[1], rel=1e-13)
            assert np.abs(b[2] - a[2]).max() <= 1e-13


@pytest.mark.parametrize("kappa", [0.2, 0.5])
def test_sound_speed_is_sqrt_kappa(kappa):
    """A small pressure pulse in a P = kappa e fluid moves at sqrt(kappa)."""
    L = 480
    z = np.arange(L) + 0.5
    z0 = L / 2
    s = ri.shock_tube(nz=L, e_L=1.0, e_R=1.0, tau=0.55)
    s.bc = ((0, 0), (0, 0), (0, 0))
    s.e0 = 1.0 + 1e-4 * np.exp(-((z - z0) ** 2) / (2 * 5.0 ** 2))
    s.n0 = s.e0 ** 0.75
    p = problem(s)
    p.kappa = kappa
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    steps = int(round(120 / math.sqrt(kappa)))
    oracle.run(p, S, steps)
    e = oracle.moments(p, S)[1] - 1.0
    right = z > z0
    centroid = (e[right] * z[right]).sum() / e[right].sum()
    assert centroid - z0 == pytest.approx(steps * math.sqrt(kappa), rel=1e-2)


def test_general_eos_conserves_and_keeps_rest_state():
    s = ri.random_state_setup(7, 6, 5, seed=24, tau=[0.8])
    p = problem(s)
    p.kappa = 0.45
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    s0 = oracle.moments(p, S)[3]
    assert oracle.run(p, S, 100) == 0
    s1 = oracle.moments(p, S)[3]
    assert np.allclose(s1[:, :2], s0[:, :2], rtol=1e-12)
    assert np.abs(s1[:, 2:] - s0[:, 2:]).max() <= 1e-12 * np.abs(s0[:, 1]).max()
    rest = oracle.Problem(4, 3, 5, tau=(0.7,), kappa=0.45)
    C = rest.cells
    R = oracle.init(rest, np.full(C, 0.8), np.full(C, 1.3), np.zeros((3, C)))
    R0 = R.copy()
    oracle.run(rest, R, 200)
    assert np.abs(R - R0).max() <= 1e-14


def test_general_eos_reverse_sweep_matches_complex_step():
    s = ri.random_state_setup(6, 5, 6, seed=25, tau=[0.75],
                              bc=((ri.INFLOW, ri.OUTFLOW), (0, 0), (ri.OUTFLOW, ri.OUTFLOW)),
                              inflow=(1.0, 1.1, 0.1, 0.0, 0.0))
    p = problem(s)
    p.kappa = 0.25
    rng = np.random.default_rng(26)
    C = s.cells
    Lo = oracle.Loss(a=rng.uniform(0.5, 1.5, C), t=rng.uniform(0.2, 1.0, C))
    G = oracle.gradient(p, s.e0, s.beta0, 10, Lo)
    v = rng.standard_normal(C) * 0.1
    _, cs = oracle.loss_cs(p, s.e0, s.beta0, 10, Lo, d_e0=v, d_tau=np.ones(1),
                           d_inflow=np.array([0.3, 0.1, -0.2, 0.05]))
    want = G.e0 @ v + G.tau[0] + G.e_in * 0.3 + G.beta_in @ np.array([0.1, -0.2, 0.05])
    assert want == pytest.approx(cs, rel=1e-9)


def test_stiff_eos_needs_a_lattice_faster_than_sound():
    """kappa = 1 gives sound speed c: at c_l = 1 it equals the lattice speed and
    the scheme goes unphysical within 30 steps on a mildly perturbed state; at
    c_l = 2 the same run stays physical."""
    for c_l, ok in ((1.0, False), (2.0, True)):
        s = ri.random_state_setup(9, 7, 8, seed=27, tau=[0.8], c_l=c_l)
        p = problem(s)
        p.kappa = 1.0
        S = oracle.init(p, s.n0, s.e0, s.beta0)
        assert (oracle.run(p, S, 30) == 0) == ok, c_l
