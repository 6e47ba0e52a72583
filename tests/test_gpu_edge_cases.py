"""Degenerate and edge cases of the GPU path against the FP64 oracle (1e-12):
one-cell lattices, the minimum extent of a non-periodic axis, lattices made
only of boundary cells, a cell walled in by solids, many one-cell instances
(ragged last workgroup), sizes one cell past a workgroup or brick, and zero
steps."""
import numpy as np
import pytest
import torch

import oracle
import rlb_inputs as ri
from helpers import fluid_mask, problem
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def test_single_cell_periodic():
    """Every pull of a 1 x 1 x 1 periodic lattice returns to the cell: pure
    relaxation towards the equilibrium of its own moments."""
    s = ri.random_state_setup(1, 1, 1, seed=601, tau=[0.8], beta_max=0.3)
    compare(s, 20)


def test_minimum_extent_outflow_axis():
    """Non-periodic axes need two cells; 1 x 1 x 2 with outflow on both faces."""
    s = ri.random_state_setup(1, 1, 2, seed=602, tau=[0.7],
                              bc=((0, 0), (0, 0), (ri.OUTFLOW, ri.OUTFLOW)))
    compare(s, 20)


def test_lattice_of_boundary_cells_only():
    """2 x 2 x 2: inflow plane and outflow plane only, plus an outflow axis."""
    s = ri.random_state_setup(2, 2, 2, seed=603, tau=[0.75],
                              bc=((ri.INFLOW, ri.OUTFLOW), (ri.OUTFLOW, ri.OUTFLOW), (0, 0)),
                              inflow=(1.0, 1.1, 0.1, 0.02, 0.0))
    compare(s, 15)


def test_cell_walled_in_by_solids():
    """3 x 3 x 3 periodic, all solid but the centre: every pull bounces back."""
    s = ri.random_state_setup(3, 3, 3, seed=604, tau=[0.9])
    solid = np.ones(27, np.uint8)
    solid[13] = 0
    s.solid = solid
    compare(s, 10)


def test_many_single_cell_instances_ragged():
    """70 instances of 1 x 1 x 1 (one workgroup plus a 6-cell ragged tail)
    with their own tau."""
    rng = np.random.default_rng(605)
    s = ri.random_state_setup(1, 1, 1, batch=70, seed=605, tau=list(rng.uniform(0.55, 1.5, 70)))
    compare(s, 12)


@pytest.mark.parametrize("n", [257, 65])
def test_one_past_a_workgroup_or_brick(n):
    s = ri.random_state_setup(n, 1, 1, seed=606, tau=[0.66],
                              bc=((ri.OUTFLOW, ri.OUTFLOW), (0, 0), (0, 0)))
    compare(s, 25)


def test_zero_steps_keeps_the_initial_fields():
    from paper_0912_2913_amd.solver import Solver

    s = ri.random_state_setup(9, 5, 7, seed=607, tau=[0.8],
                              bc=((ri.INFLOW, ri.OUTFLOW), (0, 0), (0, 0)),
                              inflow=(1.0, 1.2, 0.1, 0.0, 0.0), solid_centre=(4, 2, 3),
                              solid_radius=1.5)
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    n, e, b, _ = oracle.moments(p, S)
    sv = Solver(s)
    before = sv.state().clone()
    sv.step(0)
    assert torch.equal(sv.state(), before)
    gn, ge, gb = [x.cpu().numpy() for x in sv.moments()]
    m = fluid_mask(s)
    assert np.abs(ge[m] - e[m]).max() <= 1e-14 * np.abs(e[m]).max()
    assert np.abs(gb[:, m] - b[:, m]).max() <= 1e-14
    # a reverse sweep of zero steps returns its input buffer untouched
    seq = sv.new_g_seq(1)
    la, lb = sv.new_lam().fill_(3.0), sv.new_lam().fill_(5.0)
    assert sv.adjoint_sweep(seq, 0, la, lb) is la
    assert bool((la == 3.0).all()) and bool((lb == 5.0).all())
    sv.close()
