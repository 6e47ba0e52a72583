"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
printed constants, the analytic relativistic moments (the targets of the
paper's moment matching), conservation laws, invariant states, an independent
lumped 1-D implementation, and the exact ideal Riemann solution.
"""
import math
import os

import numpy as np
import pytest

import oracle
import rlb_inputs as ri
from oracle import d1q3

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        k, v = [s.strip() for s in line.split("=", 1)]
        try:
            out[k] = float(v)
        except ValueError:
            out[k] = v
    return out


def problem(s: ri.Setup) -> oracle.Problem:
    return oracle.Problem(s.nx, s.ny, s.nz, s.batch, s.c_l, s.bc, s.inflow, s.tau, s.solid)


# --------------------------------------------------------------------------- lattice
def test_lattice_matches_paper_constants():
    g = golden()
    e, w, opp = oracle.lattice()
    assert e.shape[0] == int(g["n_directions"])
    speeds = np.sqrt((e ** 2).sum(1))
    assert speeds.max() == pytest.approx(g["max_speed_over_c_l"], rel=1e-15)
    for q in range(19):
        s2 = int((e[q] ** 2).sum())
        want = {0: g["w_rest"], 1: g["w_axis"], 2: g["w_diag"]}[s2]
        assert w[q] == pytest.approx(want, rel=1e-15)
        assert np.all(e[opp[q]] == -e[q])
    # each velocity appears once; the lattice is D3Q19 (no (1,1,1) corners)
    assert len({tuple(v) for v in e}) == 19
    assert np.all((e ** 2).sum(1) <= 2)
    # isotropy of the weights: sum w = 1, sum w e_a e_b = delta/3,
    # sum w e_a e_b e_c e_d = (delta delta + ...)/9
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(np.einsum("q,qa,qb->ab", w, e, e), np.eye(3) / 3, atol=1e-15)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("q,qa,qb,qc,qd->abcd", w, e, e, e, e), iso4, atol=1e-15)


# --------------------------------------------------------------------------- P-1
@pytest.mark.parametrize("c_l", [1.0, 2.0, 10.0])
def test_equilibrium_moments_equal_relativistic_moments(c_l):
    """Moments of f^eq, g^eq equal N^mu = (n gamma, n gamma beta) and
    T^{mu nu} = P eta^{mu nu} + (e+P) u^mu u^nu with P = e/3 (including the
    spatial block P delta_ij + (e+P) gamma^2 beta_i beta_j)."""
    rng = np.random.default_rng(11)
    e, w, _ = oracle.lattice()
    c = c_l * e
    for _ in range(40):
        v = rng.standard_normal(3)
        beta = v / np.linalg.norm(v) * rng.uniform(0.0, 0.9)
        n, eps = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0)
        feq, geq = oracle.equilibria(n, eps, beta, c_l)
        g2 = 1.0 / (1.0 - beta @ beta)
        P = eps / 3.0
        W = (eps + P) * g2
        scale = W
        assert abs(feq.sum() - n * math.sqrt(g2)) <= 1e-14 * n * math.sqrt(g2)
        assert np.abs(feq @ c - n * math.sqrt(g2) * beta).max() <= 1e-14 * n * math.sqrt(g2) * c_l
        assert abs(geq.sum() - (W - P)) <= 1e-14 * scale
        assert np.abs(geq @ c - W * beta).max() <= 1e-14 * scale * c_l
        T_ij = np.einsum("q,qa,qb->ab", geq, c, c)
        assert np.abs(T_ij - (P * np.eye(3) + W * np.outer(beta, beta))).max() <= 1e-14 * scale * c_l ** 2


def test_equilibrium_rest_state_is_weighted():
    """At rest g^eq_i = w_i e / c_l^2 (i > 0) and f^eq_i = w_i n."""
    e, w, _ = oracle.lattice()
    for c_l in (1.0, 3.0):
        feq, geq = oracle.equilibria(0.7, 1.3, np.zeros(3), c_l)
        assert np.allclose(feq, 0.7 * w, rtol=1e-15, atol=0)
        assert np.allclose(geq[1:], 1.3 * w[1:] / c_l ** 2, rtol=1e-15, atol=0)
        assert geq[0] == pytest.approx(w[0] * 1.3 * (3 - 2 / c_l ** 2), rel=1e-15)


# --------------------------------------------------------------------------- P-2
def test_inversion_round_trip():
    """(n, e, beta) -> moments of the equilibria -> inversion -> (n, e, beta)."""
    rng = np.random.default_rng(12)
    e, _, _ = oracle.lattice()
    worst = 0.0
    for c_l in (1.0, 2.0, 10.0):
        for _ in range(60):
            v = rng.standard_normal(3)
            beta = v / np.linalg.norm(v) * rng.uniform(0.0, 0.9)
            n, eps = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0)
            feq, geq = oracle.equilibria(n, eps, beta, c_l)
            nn, ee, bb, ok = oracle.invert(feq.sum(), geq.sum(), geq @ (c_l * e))
            assert ok
            worst = max(worst, abs(nn - n) / n, abs(ee - eps) / eps, np.abs(bb - beta).max())
    assert worst <= 1e-13


def test_inversion_flags_unphysical():
    # |M| > E has no real solution; the oracle reports it and does not clamp
    n, eps, beta, ok = oracle.invert(1.0, 1.0, np.array([1.2, 0.0, 0.0]))
    assert not ok and math.isnan(eps)
    n, eps, beta, ok = oracle.invert(1.0, 1.0, np.array([0.3, 0.1, 0.0]))
    assert ok and eps > 0


# --------------------------------------------------------------------------- P-3, P-4
def test_collision_fixed_point_and_conservation():
    rng = np.random.default_rng(13)
    e, _, _ = oracle.lattice()
    for c_l in (1.0, 2.0):
        for _ in range(30):
            beta = rng.uniform(-0.25, 0.25, 3)
            n, eps = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
            feq, geq = oracle.equilibria(n, eps, beta, c_l)
            tau = rng.uniform(0.51, 2.0)
            of, og, ok = oracle.collide(feq, geq, tau, c_l)
            assert ok
            assert np.abs(of - feq).max() <= 1e-15 * np.abs(feq).max() * 4
            assert np.abs(og - geq).max() <= 1e-15 * np.abs(geq).max() * 4
            # perturbed populations: Sum f, Sum g, Sum g c conserved by the collision
            pf = feq * (1 + 0.05 * rng.standard_normal(19))
            pg = geq * (1 + 0.05 * rng.standard_normal(19))
            of, og, ok = oracle.collide(pf, pg, tau, c_l)
            assert ok
            assert abs(of.sum() - pf.sum()) <= 1e-15 * 8 * pf.sum()
            assert abs(og.sum() - pg.sum()) <= 1e-15 * 8 * pg.sum()
            assert np.abs(og @ (c_l * e) - pg @ (c_l * e)).max() <= 1e-14 * pg.sum() * c_l


def test_global_conservation_periodic():
    """Periodic box, 200 steps: Sum f, Sum g and Sum g c over the lattice are conserved."""
    s = ri.random_state_setup(6, 5, 7, seed=3, tau=[0.8])
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    _, _, _, s0 = oracle.moments(p, S)
    assert oracle.run(p, S, 200) == 0
    _, _, _, s1 = oracle.moments(p, S)
    assert abs(s1[0, 0] - s0[0, 0]) <= 1e-12 * abs(s0[0, 0])
    assert abs(s1[0, 1] - s0[0, 1]) <= 1e-12 * abs(s0[0, 1])
    assert np.abs(s1[0, 2:] - s0[0, 2:]).max() <= 1e-12 * abs(s0[0, 1])


def test_bounce_back_conserves_number_and_energy():
    """A closed periodic box with a solid ball: half-way bounce-back returns every
    population, so Sum f and Sum g over fluid cells stay constant (momentum does not)."""
    s = ri.random_state_setup(9, 8, 10, seed=4, tau=[0.7], solid_centre=(4, 4, 5), solid_radius=2.5)
    assert s.solid.sum() > 20
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    _, _, _, s0 = oracle.moments(p, S)
    oracle.run(p, S, 150)
    _, _, _, s1 = oracle.moments(p, S)
    assert abs(s1[0, 0] - s0[0, 0]) <= 1e-12 * abs(s0[0, 0])
    assert abs(s1[0, 1] - s0[0, 1]) <= 1e-12 * abs(s0[0, 1])


# --------------------------------------------------------------------------- P-5, P-6
def test_rest_state_invariance_with_obstacle():
    s = ri.random_state_setup(8, 7, 9, seed=5, tau=[0.6], solid_centre=(3, 3, 4), solid_radius=2)
    s.e0[:] = 0.8
    s.n0[:] = 0.5
    s.beta0[:] = 0.0
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    S0 = S.copy()
    oracle.run(p, S, 300)
    assert np.abs(S - S0).max() <= 1e-14 * np.abs(S0).max()


@pytest.mark.parametrize("c_l", [1.0, 2.0])
def test_uniform_flow_invariance(c_l):
    s = ri.random_state_setup(5, 4, 6, seed=6, tau=[0.7], c_l=c_l)
    s.e0[:] = 1.1
    s.n0[:] = 0.9
    s.beta0[:] = np.array([0.1, -0.05, 0.08])[:, None]
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    S0 = S.copy()
    oracle.run(p, S, 300)
    assert np.abs(S - S0).max() <= 1e-13 * np.abs(S0).max()


def test_uniform_flow_with_inflow_and_outflow_is_steady():
    """Inflow face at the interior state, outflow at the far face: a uniform flow
    along x stays uniform (pins the inflow hold and the outflow clamp)."""
    beta = (0.2, 0.0, 0.0)
    s = ri.random_state_setup(
        12, 4, 5, seed=7, tau=[0.65],
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
        inflow=(0.9, 1.1) + beta)
    s.e0[:] = 1.1
    s.n0[:] = 0.9
    s.beta0[:] = np.array(beta)[:, None]
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    S0 = S.copy()
    oracle.run(p, S, 200)
    assert np.abs(S - S0).max() <= 1e-13 * np.abs(S0).max()


def test_inflow_plane_holds_the_inflow_state():
    """A random interior next to an inflow face in a different state: the face
    cells keep the inflow state's fields (n, e, beta) at every step."""
    inflow = (0.9, 1.2, 0.15, 0.02, 0.0)
    s = ri.random_state_setup(
        9, 5, 6, seed=17, tau=[0.7],
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.PERIODIC, ri.PERIODIC)),
        inflow=inflow)
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    face = (np.arange(s.cells) % s.nx) == 0
    for _ in range(3):
        oracle.run(p, S, 7)
        n, e, b, _ = oracle.moments(p, S)
        assert np.allclose(e[face], inflow[1], rtol=1e-13, atol=0)
        assert np.allclose(n[face], inflow[0], rtol=1e-13, atol=0)
        assert np.allclose(b[:, face], np.array(inflow[2:])[:, None], rtol=0, atol=1e-14)
        assert np.abs(e[~face] - inflow[1]).max() > 1e-3  # the interior is another state


# --------------------------------------------------------------------------- P-7
@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_d3q19_line_equals_lumped_d1q3(bc):
    """On 1 x 1 x N the D3Q19 oracle must equal the independent lumped D1Q3 scheme."""
    s = ri.shock_tube(nz=160, e_L=1.0, e_R=0.40999, tau=0.58, steps=150)
    if bc == "periodic":
        s.bc = ((0, 0), (0, 0), (0, 0))
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, s.steps)
    n, e, b, _ = oracle.moments(p, S)
    n1, e1, b1 = d1q3.run(s.n0, s.e0, s.beta0[2], 0.58, 1.0, s.steps, bc=bc)
    assert np.abs(e - e1).max() <= 1e-13
    assert np.abs(b[2] - b1).max() <= 1e-13
    assert np.abs(b[:2]).max() <= 1e-15
    assert np.abs(n - n1).max() <= 1e-12  # f stays positive at this pressure ratio


def test_d3q19_line_equals_lumped_d1q3_tachyon():
    """Same equivalence at c_l = 2 (exercises every c_l factor)."""
    s = ri.shock_tube(nz=96, e_L=1.0, e_R=0.5, tau=0.7, steps=80, c_l=2.0)
    s.beta0[2][:] = 0.05
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, s.steps)
    n, e, b, _ = oracle.moments(p, S)
    n1, e1, b1 = d1q3.run(s.n0, s.e0, s.beta0[2], 0.7, 2.0, s.steps)
    assert np.abs(e - e1).max() <= 1e-13
    assert np.abs(b[2] - b1).max() <= 1e-13
    assert np.abs(n - n1).max() <= 1e-12


# --------------------------------------------------------------------------- P-9
def shear_decay_rate(L, tau, c_l, settle, steps):
    """Measured decay rate per step of beta_y = A sin(2 pi z / L) (mode
    projection after `settle` steps and after `steps` more)."""
    s = ri.shock_tube(nz=L, e_L=1.0, e_R=1.0, tau=tau, c_l=c_l)
    s.bc = ((0, 0), (0, 0), (0, 0))
    z = np.arange(L)
    s.beta0[1] = 1e-4 * np.sin(2 * np.pi * z / L)
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    mode = np.sin(2 * np.pi * z / L)
    oracle.run(p, S, settle)
    a1 = oracle.moments(p, S)[2][1] @ mode
    oracle.run(p, S, steps)
    a2 = oracle.moments(p, S)[2][1] @ mode
    return -math.log(a2 / a1) / steps


@pytest.mark.parametrize("tau,c_l", [(0.8, 1.0), (0.6, 1.0), (0.8, 2.0), (1.2, 2.0)])
def test_shear_wave_decay_matches_viscosity(tau, c_l):
    """beta_y = A sin(2 pi z / L) decays as exp(-nu k^2 t); from the paper's
    eta = (4/9) gamma^2 e (tau - dt/2) c_l^2 and (e + P) gamma^2 = (4/3) e gamma^2,
    nu = eta / ((e + P) gamma^2) = c_l^2 (tau - 1/2) dt / 3 (gamma -> 1).  With
    dx = 1 and dt = 1/c_l the decay per step is exp(-(tau - 1/2)(2 pi / L)^2 / 3).
    At L = 256 the measured rate is within 2e-4 of it, and the lattice's own
    error is second order in k: halving k (L = 128 -> 256, the same number of
    decay times) divides it by 4."""
    want = lambda L: (tau - 0.5) * (2 * np.pi / L) ** 2 / 3
    e128 = shear_decay_rate(128, tau, c_l, 200, 800) / want(128) - 1
    e256 = shear_decay_rate(256, tau, c_l, 800, 3200) / want(256) - 1
    assert abs(e256) < 2e-4
    assert 3.6 < e128 / e256 < 4.4


# --------------------------------------------------------------------------- P-10
@pytest.mark.parametrize("c_l", [1.0, 2.0])
def test_sound_speed_is_one_over_sqrt3(c_l):
    """A small pressure pulse moves at c_s = 1/sqrt(3) (units of c), i.e.
    steps * c_s / c_l cells, whatever c_l."""
    L = 480
    z = np.arange(L) + 0.5
    z0 = L / 2
    s = ri.shock_tube(nz=L, e_L=1.0, e_R=1.0, tau=0.55, c_l=c_l)
    s.bc = ((0, 0), (0, 0), (0, 0))
    s.e0 = 1.0 + 1e-4 * np.exp(-((z - z0) ** 2) / (2 * 5.0 ** 2))
    s.n0 = s.e0 ** 0.75
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    steps = int(round(120 * c_l * math.sqrt(3)))
    oracle.run(p, S, steps)
    e = oracle.moments(p, S)[1] - 1.0
    right = z > z0
    centroid = (e[right] * z[right]).sum() / e[right].sum()
    travelled = centroid - z0
    assert travelled == pytest.approx(steps / (math.sqrt(3) * c_l), rel=1e-2)


# --------------------------------------------------------------------------- step logic
@pytest.mark.parametrize("kappa,c_l", [(1.0 / 3.0, 1.0), (1.0 / 3.0, 2.0), (0.25, 1.0),
                                        (0.25, 2.0)])
def test_update_cells_equals_full_step(kappa, c_l):
    """The sampled-cell step equals the full step for either equation of state
    (P = e/3 and P = kappa e, eqs. equil2a/equil2b) and lattice speed."""
    s = ri.random_state_setup(
        7, 6, 9, batch=2, seed=8, c_l=c_l,
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
        inflow=(1.0, 1.0, 0.1, 0.0, 0.0), solid_centre=(3, 3, 4), solid_radius=1.5)
    p = oracle.Problem(s.nx, s.ny, s.nz, s.batch, s.c_l, s.bc, s.inflow, s.tau, s.solid,
                       kappa=kappa)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    S1 = S.copy()
    oracle.run(p, S1, 1)
    idx = np.arange(p.cells)
    out = oracle.update_cells(p, S, idx)
    ref = np.concatenate([S1[0], S1[1]], axis=0).T
    assert np.array_equal(out, ref)


def test_unphysical_update_is_counted():
    s = ri.random_state_setup(4, 4, 4, seed=9, tau=[0.7])
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    # one cell's +x energy population made huge: |M| > E at the cell it streams to
    S[1, 1, 5] = 50.0
    S[1, 2, 5] = -40.0
    bad = oracle.run(p, S, 1)
    assert bad >= 1
