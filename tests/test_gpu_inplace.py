"""In-place (AA-pattern) streaming against the FP64 oracle's two-buffer pull
steps: one state buffer, the same results (FP64 at the 1e-12 bar) after
every even number of steps, for every boundary kind."""
import numpy as np
import pytest
import torch

import oracle
import rlb_inputs as ri
from helpers import problem
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def same_bits(a: torch.Tensor, b: torch.Tensor) -> bool:
    """Bitwise equality (NaN payloads included: the sphere goes unphysical)."""
    return torch.equal(a.contiguous().view(torch.uint8), b.contiguous().view(torch.uint8))


def inplace(s):
    s.inplace = True
    return s


CASES = {
    "periodic_batch": lambda: ri.random_state_setup(9, 7, 8, batch=3, seed=701,
                                                    tau=[0.55, 0.9, 1.4]),
    "outflow_all_faces": lambda: ri.random_state_setup(8, 6, 7, seed=702, tau=[0.8],
                                                       bc=((1, 1), (1, 1), (1, 1))),
    "inflow_outflow_obstacle": lambda: ri.random_state_setup(
        13, 7, 9, batch=2, seed=703, tau=[0.65, 0.9],
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
        inflow=(1.0, 1.05, 0.15, 0.03, -0.02), solid_centre=(6, 3, 4), solid_radius=2.2),
    "solid_on_outflow_face": lambda: ri.random_state_setup(
        8, 9, 7, seed=704, tau=[0.75],
        bc=((ri.OUTFLOW, ri.INFLOW), (ri.OUTFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC)),
        inflow=(1.0, 0.95, -0.1, 0.05, 0.0), solid_centre=(0, 4, 3), solid_radius=2.0),
    "tachyon": lambda: ri.random_state_setup(6, 7, 5, seed=705, tau=[0.9], c_l=2.0,
                                             bc=((0, 0), (1, 1), (0, 0))),
    "minimal_boundary_only": lambda: ri.random_state_setup(
        2, 2, 2, seed=706, tau=[0.75], bc=((ri.INFLOW, ri.OUTFLOW), (1, 1), (0, 0)),
        inflow=(1.0, 1.1, 0.1, 0.02, 0.0)),
    "tube": lambda: ri.shock_tube(nz=200, e_L=1.0, e_R=0.40999, tau=0.6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_inplace_matches_oracle(name):
    compare(inplace(CASES[name]()), 30)


@pytest.mark.parametrize("kappa,c_l", [(0.25, 1.0), (0.7, 2.0)])
def test_inplace_general_eos_matches_oracle(kappa, c_l):
    """P = kappa e with in-place streaming, every boundary kind and an
    obstacle, against the oracle's two-buffer steps at 1e-12."""
    s = CASES["inflow_outflow_obstacle"]()
    s.kappa = kappa
    s.c_l = c_l
    compare(inplace(s), 30)


def test_inplace_small_sphere_matches_oracle():
    """30 x 20 x 20 sphere set-up (inflow |beta| = 0.5, outflow, obstacle of
    radius 4), 20 steps, against the oracle."""
    compare(inplace(ri.sphere(nx=30, ny=20, nz=20, centre=(12, 10, 10), radius=4)), 20)


def test_inplace_sphere_block_against_two_buffer_run():
    """A 60 x 40 x 40 sphere over 40 steps (it goes unphysical on the way, as
    the published scheme does at c_l = 1).  Over the first 12 steps, while
    the fields are still smooth, the in-place and two-buffer GPU runs agree
    to 1e-12 at every other step.  Later the state is chaotic: a last-bit
    difference between two differently compiled kernels grows by orders of
    magnitude (measured between two builds of the two-buffer step kernel:
    the first differing values, at step 16, differ by 2e-15; by step 40 by
    up to 6e-9).  There the runs must have the same unphysical and
    f-positivity counts after every pair of steps, the same NaN cells at the
    end, and agree to 1e-6."""
    from paper_0912_2913_amd.solver import Solver

    mk = lambda: ri.sphere(nx=60, ny=40, nz=40, centre=(20, 20, 20), radius=6)
    a = Solver(mk())
    b = Solver(inplace(mk()))
    ca, cb = np.zeros(2, np.int64), np.zeros(2, np.int64)
    for step in range(2, 41, 2):  # the in-place state reads back after even step counts
        a.step(2)
        b.step(2)
        ca += a.counters()
        cb += b.counters()
        assert tuple(ca) == tuple(cb), step
        if step <= 12:
            x, y = a.populations(), b.populations()
            assert torch.allclose(x, y, rtol=1e-12, atol=1e-300), step
    assert ca[0] > 0  # the run did go unphysical
    x, y = a.populations(), b.populations()
    assert torch.equal(torch.isnan(x), torch.isnan(y))
    f = ~torch.isnan(x)
    assert torch.allclose(x[f], y[f], rtol=1e-6, atol=1e-300)
    assert len(b.pop) == 1  # one state buffer
    a.close()
    b.close()


@pytest.mark.parametrize("collide", [ri.COLLIDE_AUTO, ri.COLLIDE_F32_MOM64])
def test_inplace_fp32_deviation_storage_matches_two_buffer_run(collide):
    from paper_0912_2913_amd.solver import Solver

    mk = lambda: CASES["inflow_outflow_obstacle"]().with_(storage=ri.F32DEV, collide=collide)
    a = Solver(mk())
    a.step(20)
    b = Solver(inplace(mk()))
    b.step(20)
    assert same_bits(a.populations(), b.populations())
    a.close()
    b.close()


def test_inplace_odd_step_count_and_unavailable_entry_points():
    from paper_0912_2913_amd._lib import RLBError
    from paper_0912_2913_amd.solver import Solver

    s = inplace(CASES["inflow_outflow_obstacle"]())
    sv = Solver(s)
    sv.step(3)
    with pytest.raises(RLBError):
        sv.moments()
    with pytest.raises(RLBError):
        sv.transport()
    sv.step(1)
    sv.moments()
    g = torch.empty((sv.nbrick, 19, 64), dtype=sv.dtype, device=sv.device)
    with pytest.raises(RLBError):
        sv.step_g(sv.state()[1], g)
    with pytest.raises(RLBError):
        sv.hold_eta_over_s(0.1)
    lam = sv.new_lam().zero_()
    with pytest.raises(RLBError):
        sv.adjoint_step(sv.state()[1], lam, sv.new_lam())
    sv.set_tau_field(np.full(s.cells, 0.8))  # a tau field works in place
    sv.step(2)
    sv.close()
