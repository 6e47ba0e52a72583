"""General equation of state P = kappa e on the GPU (eqs. equil1, equil2a,
equil2b and the matching inversion) against the FP64 oracle, through the C
ABI: FP64 at the 1e-12 bar, the FP32-deviation storage at its own bound; the
reverse mode per entry point at 1e-12 and the checkpointed gradient at 1e-10,
as for e = 3P."""
import numpy as np
import pytest
import torch

import oracle
import rlb_inputs as ri
from helpers import field_err, fluid_mask, oracle_fields, problem
from test_gpu_adjoint import _gpu_gradient, _loss_arrays, rel, upload_g, upload_lam
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def obstacle_setup(seed, kappa, storage=ri.F64):
    s = ri.random_state_setup(
        13, 7, 9, batch=2, seed=seed, tau=[0.65, 0.9],
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
        inflow=(1.0, 1.05, 0.15, 0.03, -0.02), solid_centre=(6, 3, 4), solid_radius=2.2,
        storage=storage)
    s.kappa = kappa
    return s


@pytest.mark.parametrize("kappa,c_l", [(0.2, 1.0), (0.6, 1.0), (1.0, 2.0)])
def test_general_eos_forward_matches_oracle(kappa, c_l):
    """kappa = 1 (sound speed c) runs at c_l = 2: at c_l = 1 the sound speed
    reaches the lattice speed and the scheme itself goes unphysical."""
    s = obstacle_setup(501, kappa)
    s.c_l = c_l
    compare(s, 30)


def test_general_eos_periodic_batch_tachyon():
    s = ri.random_state_setup(9, 8, 11, batch=2, seed=502, tau=[0.7, 1.1], c_l=2.0)
    s.kappa = 0.25
    compare(s, 30)


def test_general_eos_fp32_deviation_storage():
    """FP32 deviations from the rest state of the same EoS (FP64 collision):
    the per-step rounding is ~1e-7 of the deviations, so e and beta stay
    within 2e-6 of the FP64 oracle over 20 steps."""
    from paper_0912_2913_amd.solver import Solver

    s = obstacle_setup(503, 0.45, storage=ri.F32DEV)
    _, e, b, _, _, _ = oracle_fields(s, 20)
    sv = Solver(s)
    sv.step(20)
    _, ge, gb = [x.cpu().numpy() for x in sv.moments()]
    m = fluid_mask(s)
    assert field_err(ge, e, m) <= 2e-6
    assert np.abs(gb[:, m] - b[:, m]).max() <= 2e-6 * np.abs(b[:, m]).max()
    sv.close()


def test_general_eos_rejects_the_e_3p_only_transport_rules():
    from paper_0912_2913_amd._lib import RLBError
    from paper_0912_2913_amd.solver import Solver

    for bad in (1.5, -0.1):
        with pytest.raises(RLBError):
            Solver(obstacle_setup(504, bad))
    s = obstacle_setup(504, 0.3)
    sv = Solver(s)
    with pytest.raises(RLBError):
        sv.transport()
    with pytest.raises(RLBError):
        sv.hold_eta_over_s(0.1)
    sv.step_g(sv.g_state(), sv.new_g())  # the g-only forward step is EoS-general
    sv.close()


@pytest.mark.parametrize("kappa,c_l", [(0.2, 1.0), (0.6, 1.0), (1.0, 2.0)])
def test_general_eos_adjoint_entry_points_match_oracle(kappa, c_l):
    """rlb_adjoint_step, rlb_moments_adjoint and rlb_init_adjoint with the
    general equilibria and inversion, element by element against the
    oracle's complex-step transposes."""
    from paper_0912_2913_amd.solver import Solver

    s = obstacle_setup(505, kappa)
    s.c_l = c_l
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, 3)
    Sg = np.ascontiguousarray(S[1])
    rng = np.random.default_rng(506)
    lam = rng.standard_normal(Sg.shape)
    lam_t, dtau, dbin, dein = oracle.adjoint_step(p, Sg, lam)
    sv = Solver(s)
    lo = torch.full_like(upload_lam(sv, lam), float("nan"))
    dt = torch.zeros(s.batch, dtype=torch.float64, device=sv.device)
    db = torch.zeros(3, dtype=torch.float64, device=sv.device)
    de = torch.zeros(1, dtype=torch.float64, device=sv.device)
    sv.adjoint_step(upload_g(sv, Sg), upload_lam(sv, lam), lo, dt, db, de)
    got = sv.unpack(lo).cpu().numpy()
    assert np.isfinite(got).all()
    assert rel(got, lam_t) <= 1e-12
    assert rel(dt.cpu().numpy(), dtau) <= 1e-12
    assert rel(db.cpu().numpy(), dbin) <= 1e-12
    assert rel(de.cpu().numpy(), np.array([dein])) <= 1e-12

    dLde = rng.standard_normal(s.cells)
    dLdb = rng.standard_normal((3, s.cells))
    lam_ref = oracle.moments_adjoint(p, Sg, dLde, dLdb)
    lm = sv.new_lam()
    sv.moments_adjoint(upload_g(sv, Sg), torch.as_tensor(dLde, device=sv.device),
                       torch.as_tensor(dLdb, device=sv.device), lm)
    assert rel(sv.unpack(lm).cpu().numpy(), lam_ref) <= 1e-12

    lam0 = rng.standard_normal((19, s.cells))
    de0_ref, db0_ref, dbin_ref, dein_ref = oracle.init_adjoint(p, s.e0, s.beta0, lam0)
    de0 = torch.empty(s.cells, dtype=torch.float64, device=sv.device)
    db0 = torch.empty((3, s.cells), dtype=torch.float64, device=sv.device)
    dbi = torch.zeros(3, dtype=torch.float64, device=sv.device)
    dei = torch.zeros(1, dtype=torch.float64, device=sv.device)
    sv.init_adjoint(upload_lam(sv, lam0), de0, db0, dbi, dei)
    assert rel(de0.cpu().numpy(), de0_ref) <= 1e-12
    assert rel(db0.cpu().numpy(), db0_ref) <= 1e-12
    assert rel(dbi.cpu().numpy(), dbin_ref) <= 1e-12
    assert rel(dei.cpu().numpy(), np.array([dein_ref])) <= 1e-12
    sv.close()


@pytest.mark.parametrize("kappa,c_l", [(0.25, 1.0), (0.8, 2.0)])
def test_general_eos_checkpointed_gradient_matches_oracle(kappa, c_l):
    """The sqrt(T)-checkpointed gradient (autograd over the C ABI) of a loss on
    the final fields, against the oracle's store-all FP64 reverse sweep."""
    s = obstacle_setup(507, kappa)
    s.c_l = c_l
    steps = 25
    a, t, be, bb = _loss_arrays(s, 1)
    G = oracle.gradient(problem(s), s.e0, s.beta0, steps, oracle.Loss(a, t, be, bb))
    L, gt, gei, gbi, ge0, gb0 = _gpu_gradient(s, steps, "sqrt", seed=1)
    assert L == pytest.approx(G.loss, rel=1e-12)
    assert rel(gt, G.tau) <= 1e-10
    assert rel(ge0, G.e0) <= 1e-10
    assert rel(gb0, G.beta0) <= 1e-10
    assert rel(gbi, G.beta_in) <= 1e-10
    assert rel(gei, np.array([G.e_in])) <= 1e-10


def test_general_eos_tau_field_gradient_matches_oracle():
    """A per-cell tau field with P = kappa e: the checkpointed gradient with
    respect to tau(x) (and the instance tau) against the oracle's reverse
    sweep at 1e-10."""
    from paper_0912_2913_amd.autograd import rlb_run

    s = obstacle_setup(508, 0.3)
    s.tau_cell = np.random.default_rng(509).uniform(0.6, 1.1, s.cells)
    steps = 20
    rng = np.random.default_rng(510)
    C = s.cells
    a, t = rng.uniform(0.5, 1.5, C), rng.uniform(0.2, 1.0, C)
    G = oracle.gradient(problem(s), s.e0, s.beta0, steps, oracle.Loss(a=a, t=t))
    dev = "cuda:0"
    tau = torch.tensor(s.tau, device=dev, requires_grad=True)
    tc = torch.tensor(s.tau_cell, device=dev, requires_grad=True)
    e, _ = rlb_run(s, steps, tau=tau, tau_cell=tc)
    m = torch.as_tensor(s.solid == 0, device=dev)
    at, tt = torch.as_tensor(a, device=dev), torch.as_tensor(t, device=dev)
    L = ((at * (e - tt) ** 2)[m]).sum()
    L.backward()
    assert float(L) == pytest.approx(G.loss, rel=1e-12)
    gtc = tc.grad.cpu().numpy()
    assert np.abs(gtc - G.tau_cell).max() <= 1e-10 * np.abs(G.tau_cell).max()
    gt = tau.grad.cpu().numpy()
    assert np.abs(gt - G.tau).max() <= 1e-10 * np.abs(G.tau).max()
