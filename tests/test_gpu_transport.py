"""Per-cell relaxation times, held eta/s and transport diagnostics on the GPU
against the FP64 oracle, through the C ABI (FP64 storage, 1e-12 bar for the
forward fields, 1e-10 for gradients as in the other adjoint tests)."""
import numpy as np
import pytest
import torch

import oracle
import rlb_inputs as ri
from helpers import field_err, fluid_mask, problem
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def obstacle_setup(seed=401):
    return ri.random_state_setup(
        13, 7, 9, batch=2, seed=seed, tau=[0.65, 0.9],
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
        inflow=(1.0, 1.05, 0.15, 0.03, -0.02), solid_centre=(6, 3, 4), solid_radius=2.2)


def with_tau_field(s, seed=7, lo=0.55, hi=1.3):
    s.tau_cell = np.random.default_rng(seed).uniform(lo, hi, s.cells)
    return s


def test_tau_field_forward_matches_oracle():
    compare(with_tau_field(obstacle_setup()), 30)


def test_tau_field_periodic_batch_ragged():
    s = with_tau_field(ri.random_state_setup(11, 9, 7, batch=3, seed=402, tau=[0.6, 0.8, 1.0]), 8)
    compare(s, 25)


def test_held_eta_over_s_matches_oracle_on_the_paper_tube():
    """1 x 1 x 800 tube at the paper's pressure ratio e_R/e_L = 0.40999, 400
    steps, tau set every step from the local state to hold eta/s = 0.1."""
    s = ri.shock_tube(nz=800, e_L=1.0, e_R=0.40999, tau=0.6)
    s.eta_s = 0.1
    compare(s, 400)


def test_held_eta_over_s_matches_oracle_3d():
    s = ri.random_state_setup(10, 9, 8, batch=2, seed=403, tau=[0.7, 0.7])
    s.eta_s = 0.05
    compare(s, 30)


@pytest.mark.parametrize("mode", ["instance", "field", "eta_s"])
def test_transport_diagnostics_match_oracle(mode):
    from paper_0912_2913_amd.solver import Solver

    s = obstacle_setup(404)
    if mode == "field":
        with_tau_field(s, 9)
    if mode == "eta_s":
        s.eta_s = 0.08
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, 12)
    ref = oracle.transport(p, S)
    sv = Solver(s)
    sv.step(12)
    got = [t.cpu().numpy() for t in sv.transport(s.d_G)]
    m = fluid_mask(s)
    for name, g, r in zip(("T", "s", "eta", "eta_over_s"), got, ref):
        assert field_err(g, r, m) <= 1e-12, name
        assert np.all(g[~m] == 0.0)
    if mode == "eta_s":
        assert np.allclose(got[3][m], 0.08, rtol=1e-12)
    sv.close()


def test_tau_field_gradient_matches_oracle_reverse_sweep():
    from paper_0912_2913_amd.autograd import rlb_run

    s = with_tau_field(obstacle_setup(405), 11, 0.6, 1.1)
    steps = 20
    rng = np.random.default_rng(12)
    C = s.cells
    a, t = rng.uniform(0.5, 1.5, C), rng.uniform(0.2, 1.0, C)
    bb = rng.standard_normal((3, C)) * 0.1
    G = oracle.gradient(problem(s), s.e0, s.beta0, steps, oracle.Loss(a=a, t=t, bb=bb))
    dev = "cuda:0"
    tau = torch.tensor(s.tau, device=dev, requires_grad=True)
    tc = torch.tensor(s.tau_cell, device=dev, requires_grad=True)
    e, b = rlb_run(s, steps, tau=tau, tau_cell=tc)
    m = torch.as_tensor(s.solid == 0, device=dev)
    at, tt, bt = (torch.as_tensor(v, device=dev) for v in (a, t, bb))
    L = ((at * (e - tt) ** 2)[m]).sum() + ((bt * b)[:, m]).sum()
    L.backward()
    assert float(L) == pytest.approx(G.loss, rel=1e-12)
    gtc = tc.grad.cpu().numpy()
    assert np.abs(gtc - G.tau_cell).max() <= 1e-10 * np.abs(G.tau_cell).max()
    gt = tau.grad.cpu().numpy()
    assert np.abs(gt - G.tau).max() <= 1e-10 * np.abs(G.tau).max()


def test_tau_field_and_eta_s_reject_invalid_use():
    from paper_0912_2913_amd._lib import RLBError
    from paper_0912_2913_amd.solver import Solver

    s = obstacle_setup(406)
    sv = Solver(s)
    with pytest.raises(RLBError):
        sv.adjoint_flush_tau_field(torch.zeros(s.cells, dtype=torch.float64, device="cuda:0"))
    good = np.full(s.cells, 0.8)
    sv.set_tau_field(good)
    bad = good.copy()
    bad[np.flatnonzero(s.solid.reshape(-1) == 0)[5]] = 0.5
    with pytest.raises(RLBError):
        sv.set_tau_field(bad)
    # the previous field stays in force: the run equals one with tau = 0.8 everywhere
    sv.step(5)
    e1 = sv.moments()[1].cpu().numpy()
    s2 = obstacle_setup(406)
    s2.tau = np.array([0.8, 0.8])
    sv2 = Solver(s2)
    sv2.step(5)
    assert np.array_equal(e1, sv2.moments()[1].cpu().numpy())
    sv2.close()
    # a NaN on a solid cell is ignored (solid cells never relax)
    nan_on_solid = good.copy()
    nan_on_solid[np.flatnonzero(s.solid.reshape(-1) != 0)[0]] = np.nan
    sv.set_tau_field(nan_on_solid)
    for bad_args in ((-0.1, 16.0), (0.1, 0.0), (float("nan"), 16.0)):
        with pytest.raises(RLBError):
            sv.hold_eta_over_s(*bad_args)
    sv.hold_eta_over_s(0.1)
    g = sv.new_g()
    with pytest.raises(RLBError):
        sv.step_g(sv.g_state(), g)
    with pytest.raises(RLBError):
        sv.transport(d_G=8.0)
    sv.hold_eta_over_s(0.0)
    sv.step_g(sv.g_state(), g)
    sv.close()
