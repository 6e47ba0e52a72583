"""Failure detection and resume through the C ABI.

Unphysical states (the moment relations have no physical solution: NaN, or
|M| >= E so that e <= 0) are forced from the host into one update's pulled
populations; one step later the library's counter reports exactly that update
and rlb_counters returns RLB_EUNPHYSICAL.  A run stopped after k steps and
continued in a fresh solver from a copy of its state matches the uninterrupted
run bit for bit.
"""
import numpy as np
import pytest
import torch

import rlb_inputs as ri

pytestmark = pytest.mark.gpu

E_INT = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
         (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def _solver(s):
    from paper_0912_2913_amd.solver import Solver

    return Solver(s)


def _setup(storage=ri.F64):
    return ri.random_state_setup(12, 10, 9, seed=401, tau=[0.8], storage=storage)


def _write(sv, pop: int, q: int, cell: int, value: float):
    """Set one stored population value (brick layout) of the current state."""
    st = sv.state()
    st[pop, cell // 64, q, cell % 64] = value


def _pulled(s, cell):
    """(source cell, direction) of the 19 pulls of `cell` on a periodic box."""
    x = cell % s.nx
    y = (cell // s.nx) % s.ny
    z = cell // (s.nx * s.ny)
    out = []
    for q, (ex, ey, ez) in enumerate(E_INT):
        sx, sy, sz = (x - ex) % s.nx, (y - ey) % s.ny, (z - ez) % s.nz
        out.append(((sz * s.ny + sy) * s.nx + sx, q))
    return out


@pytest.mark.parametrize("storage", [ri.F64, ri.F32, ri.BF16DEV],
                         ids=lambda v: ri.STORAGE_NAMES[v])
def test_nan_in_one_update_is_counted(storage):
    from paper_0912_2913_amd._lib import UnphysicalState

    s = _setup(storage)
    sv = _solver(s)
    sv.step(4)
    assert sv.counters() == (0, 0)
    cell = 5 * s.nx * s.ny + 4 * s.nx + 7
    _write(sv, 1, 0, cell, float("nan"))  # the rest population is pulled by its own cell only
    sv.step(1)
    with pytest.raises(UnphysicalState):
        sv.counters(raise_on_unphysical=True)
    # the call above reset the counters; the state still holds the NaN
    sv2 = _solver(s)
    sv2.step(4)
    _write(sv2, 1, 0, cell, float("nan"))
    sv2.step(1)
    unphysical, nonpositive = sv2.counters()
    assert unphysical == 1 and nonpositive == 1
    e = sv2.moments()[1].cpu().numpy()
    assert np.isnan(e[cell]) and np.isfinite(np.delete(e, cell)).all()
    sv.close()
    sv2.close()


def test_momentum_beyond_energy_in_one_update_is_counted():
    """The 19 values one cell pulls are rewritten so that its moments have
    |M| > E (the +x mover carries +1, the -x mover -0.5, the rest 0): the
    relations give e <= 0 there, and nowhere else."""
    s = _setup()
    sv = _solver(s)
    sv.step(3)
    cell = 4 * s.nx * s.ny + 6 * s.nx + 2
    for src, q in _pulled(s, cell):
        v = 1.0 if q == 1 else (-0.5 if q == 2 else 0.0)
        _write(sv, 1, q, src, v)
    st = sv.populations().cpu().numpy()
    g = np.array([st[1, q, src] for src, q in _pulled(s, cell)])
    E = g.sum()
    M = np.array([sum(g[q] * E_INT[q][k] for q in range(19)) for k in range(3)]) * s.c_l
    assert np.linalg.norm(M) > E > 0
    sv.step(1)
    assert sv.counters()[0] == 1
    sv.close()


@pytest.mark.parametrize("storage", [ri.F64, ri.BF16DEV], ids=lambda v: ri.STORAGE_NAMES[v])
def test_resume_from_copied_state_is_bitwise(storage):
    s = ri.random_state_setup(
        15, 9, 11, seed=402, tau=[0.7], storage=storage,
        bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
        inflow=(1.0, 1.05, 0.1, 0.0, 0.0), solid_centre=(7, 4, 5), solid_radius=2.5)
    a = _solver(s)
    a.step(13)
    b = _solver(s)  # fresh solver: its current state is pop_a
    b.state().copy_(a.state())
    a.step(21)
    b.step(21)
    torch.cuda.synchronize()
    # every cell's 38 stored values, bit for bit (the padding past the last cell
    # is never written)
    pa, pb = a.populations(), b.populations()
    assert torch.equal(pa.view(torch.uint8), pb.view(torch.uint8))
    assert a.counters() == b.counters()
    a.close()
    b.close()
