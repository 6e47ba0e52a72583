"""Checkpoint schedules of the differentiable run (host logic, no GPU).

GRun drives the library through the solver's g-only entry points; here a
stand-in solver with the same calls runs a small nonlinear recurrence on the
CPU, so that every schedule can be checked for what it must do: visit the
reverse steps T-1 .. 0 once each, in order, each with the state of its own
step, and give the store-all result bit for bit; the 3-level schedule's
lengths hold about 3 T^(1/3) states.
"""
import math

import pytest
import torch

from paper_0912_2913_amd.autograd import GRun, peak_states, schedule


class RecurrenceSolver:
    """x_{t+1} = x_t + h sin(A x_t); lambda_t = lambda_{t+1} + h A^T (cos(A x_t) lambda_{t+1});
    the 'tau' partial is the step-ordered sum of lambda_{t+1} . sin(A x_t)."""

    def __init__(self, d=5, seed=0):
        g = torch.Generator().manual_seed(seed)
        self.A = torch.randn(d, d, generator=g, dtype=torch.float64) * 0.5
        self.x0 = torch.randn(d, generator=g, dtype=torch.float64)
        self.h = 0.1
        self.batch, self.cells, self.device, self.tau_cell = 1, d, "cpu", None
        self.visited = []
        self._pending = torch.zeros(1, dtype=torch.float64)

    def _step(self, x):
        return x + self.h * torch.sin(self.A @ x)

    def g_state(self):
        return self.x0

    def new_g(self):
        return torch.empty(self.cells, dtype=torch.float64)

    def new_lam(self):
        return torch.empty(self.cells, dtype=torch.float64)

    def new_g_seq(self, n):
        return torch.empty((n, self.cells), dtype=torch.float64)

    def advance_g(self, src, dst, tmp, n):
        x = src.clone()
        for _ in range(n):
            x = self._step(x)
        dst.copy_(x)

    def trajectory_g(self, seq, n):
        for i in range(1, n):
            seq[i].copy_(self._step(seq[i - 1]))

    def step_g(self, src, dst):
        dst.copy_(self._step(src))

    def adjoint_step(self, x, la, lb, dtau=None, dbin=None, dein=None):
        self.visited.append(x.clone())
        s = self.A @ x
        self._pending += (la * torch.sin(s)).sum()
        lb.copy_(la + self.h * (self.A.T @ (torch.cos(s) * la)))

    def adjoint_sweep(self, seq, n, la, lb):
        a, b = la, lb
        for i in range(n - 1, -1, -1):
            x = seq[i]
            self.visited.append(x.clone())
            s = self.A @ x
            self._pending += (a * torch.sin(s)).sum()
            b.copy_(a + self.h * (self.A.T @ (torch.cos(s) * a)))
            a, b = b, a
        return a

    # The library passes lambda between segments in a "reader form"; the stand-in
    # models it as the reversed vector, so that a schedule that forgot to
    # gather it back would fail.
    def adjoint_segment(self, g_first, g_seq, n, la, lb, in_reader=False, out_reader=False):
        states = ([g_first] + [g_seq[j] for j in range(n - 1)]) if g_first is not None \
            else [g_seq[j] for j in range(n)]
        a, b = la, lb
        reader = in_reader
        for x in reversed(states):
            lam = a.flip(0) if reader else a
            self.visited.append(x.clone())
            s = self.A @ x
            self._pending += (lam * torch.sin(s)).sum()
            b.copy_((lam + self.h * (self.A.T @ (torch.cos(s) * lam))).flip(0))
            a, b = b, a
            reader = True
        if reader and not out_reader:
            self.lam_gather(a, b)
            a, b = b, a
        return a

    def lam_gather(self, lam_reader, lam_out):
        lam_out.copy_(lam_reader.flip(0))

    def adjoint_flush(self, dtau=None, dbin=None, dein=None):
        if dtau is not None:
            dtau += self._pending
        self._pending = torch.zeros(1, dtype=torch.float64)

    def fields_g(self, g):
        return g.clone(), torch.stack([g, g, g])

    def moments_adjoint(self, g, dLde, dLdb, lam):
        lam.copy_(dLde + dLdb.sum(0))

    def init_adjoint(self, lam, de0, db0, dbin=None, dein=None):
        de0.copy_(lam)
        db0.copy_(torch.stack([lam, lam, lam]))


def run(T, mode):
    sv = RecurrenceSolver()
    r = GRun(sv, T, schedule(T, mode))
    e, _ = r.forward()
    dLde = torch.linspace(-1.0, 1.0, sv.cells, dtype=torch.float64)
    dLdb = torch.zeros((3, sv.cells), dtype=torch.float64)
    dtau, _, _, de0, _, _ = r.backward(dLde, dLdb)
    return sv, e, dtau, de0


@pytest.mark.parametrize("T", [1, 2, 7, 8, 9, 26, 27, 28, 64, 100])
@pytest.mark.parametrize("mode", ["sqrt", "3level", 5, "store_all"])
def test_schedules_visit_every_step_once_in_order_and_agree_bitwise(T, mode):
    ref_sv, ref_e, ref_tau, ref_de0 = run(T, "store_all")
    sv, e, dtau, de0 = run(T, mode)
    # the true trajectory, one state per step
    xs = [sv.x0.clone()]
    for _ in range(T):
        xs.append(sv._step(xs[-1]))
    assert torch.equal(e, xs[T])
    assert len(sv.visited) == T
    for k, x in enumerate(sv.visited):
        assert torch.equal(x, xs[T - 1 - k]), f"reverse step {k} saw the wrong state"
    assert torch.equal(dtau, ref_tau) and torch.equal(de0, ref_de0)


@pytest.mark.parametrize("T", [10, 64, 100, 1000, 2000, 4000])
def test_three_level_schedule_holds_about_three_cube_roots(T):
    l1, l2 = schedule(T, "3level")
    assert l2 ** 3 >= T > (l2 - 1) ** 3 and l1 == min(T, l2 * l2)
    p3, p2 = peak_states(T, "3level"), peak_states(T, "sqrt")
    assert p3 <= 3 * math.ceil(T ** (1.0 / 3.0)) + 1
    if T >= 64:
        assert p3 < p2


def test_schedule_lengths():
    assert schedule(4000, "sqrt") == [64]
    assert schedule(4000, "3level") == [256, 16]
    assert schedule(2000, "3level") == [169, 13]
    assert schedule(10, "store_all") == [10]
    assert schedule(10, 4) == [4]
    assert peak_states(4000, "sqrt") == 63 + 63
    assert peak_states(4000, "3level") == 16 + 16 + 15
    with pytest.raises(ValueError):
        schedule(10, "quartic")
