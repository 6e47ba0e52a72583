"""Differentiable RLB runs: a torch.autograd.Function over the library's forward
and adjoint kernels, with sqrt(T) checkpointing of the g population.

Only the energy-momentum population g enters (e, beta) (the constraint for n
involves f alone and f^eq depends on beta only), so a loss on the final (e, beta)
fields has zero derivative with respect to f and the reverse sweep runs on g
alone: every checkpoint and recomputed state is a g block in the solver's
storage format, and the recompute is bit-identical to the forward.

Schedule for T steps with segment length S (default ceil(sqrt(T))):
  forward  -- g-only steps from S_0; keep S_0, S_S, S_2S, ... (K = ceil(T/S)),
              each segment advancing straight into the next checkpoint;
  backward -- lambda_T from the moment map; for each segment from the last:
              recompute its S - 1 later states from its checkpoint (read in
              place, not copied), then run the adjoint steps down through the
              segment in one library call; lambda passes from segment to
              segment in the library's reader form (each reverse step's
              contributions stored at the cell that made them) and is gathered
              into its natural form once, before lambda_0 is mapped to the
              initial fields.
Peak storage: K checkpoints + S - 1 segment states + 2 lambda buffers.  S = T
keeps every state (store-all).

When even 2 sqrt(T) states do not fit, "3level" nests one more level: segments
of L1 = ceil(T^(2/3)) steps are split into sub-segments of L2 = ceil(T^(1/3))
steps whose checkpoints are recomputed per segment in the backward pass, so that
about 3 T^(1/3) states are held for one more g-only forward pass.  Every
schedule gives the same gradient bit for bit (the recompute is bit-identical
and the reverse partials accumulate in step order whatever the split).
"""
from __future__ import annotations

import math
from dataclasses import replace
from typing import List, Optional

import numpy as np
import torch

from .solver import Solver


# Reverse passes of the sqrt(T) schedule overlap each segment's recompute with
# the previous segment's sweep on lattices of at most this many cells (where a
# single launch leaves most of the device idle).
OVERLAP_RECOMPUTE = True
OVERLAP_MAX_CELLS = 1 << 22


def _iroot(T: int, k: int) -> int:
    """Smallest r >= 1 with r**k >= T."""
    r = max(1, int(round(T ** (1.0 / k))))
    while r ** k < T:
        r += 1
    while r > 1 and (r - 1) ** k >= T:
        r -= 1
    return r


def schedule(T: int, mode="sqrt") -> List[int]:
    """Segment lengths from the outermost level in: [S] for "sqrt" (S =
    ceil(sqrt(T))), "store_all" ([T]) or an int segment length; [L1, L2] with
    L1 = ceil(T^(2/3)) and L2 = ceil(T^(1/3)) for "3level"."""
    if T <= 0:
        return [1]
    if mode == "store_all":
        return [T]
    if isinstance(mode, int) and not isinstance(mode, bool):
        return [max(1, min(T, mode))]
    if mode == "sqrt":
        return [_iroot(T, 2)]
    if mode == "3level":
        l2 = _iroot(T, 3)
        return [min(T, l2 * l2), l2]
    raise ValueError(f"unknown checkpoint schedule {mode!r}")


def segment_length(T: int, mode="sqrt") -> int:
    return schedule(T, mode)[0]


def peak_states(T: int, mode="sqrt") -> int:
    """g states held at once by the schedule (checkpoints of every level plus
    the innermost segment's recomputed states after its checkpoint), lambda
    and ping-pong buffers excluded."""
    lens = schedule(T, mode)
    outer = [T] + lens
    n = 0
    for lv, L in enumerate(lens):
        n += (outer[lv] + L - 1) // L  # checkpoints of this level (its first is the level above's)
    return n + lens[-1] - 1


class GRun:
    """A g-only forward run of T steps on one solver with checkpoints."""

    def __init__(self, solver: Solver, T: int, seg):
        """seg: the segment length, or the list of segment lengths from the
        outermost level in (see schedule())."""
        self.sv = solver
        self.T = int(T)
        self.lens = [int(v) for v in (seg if isinstance(seg, (list, tuple)) else [seg])]
        if any(v < 1 for v in self.lens) or any(b > a for a, b in zip(self.lens, self.lens[1:])):
            raise ValueError("segment lengths must be >= 1 and non-increasing")
        self.S = self.lens[0]
        self.K = (self.T + self.S - 1) // self.S if self.T > 0 else 1
        self.ckpt: List[torch.Tensor] = []
        self.final: Optional[torch.Tensor] = None

    def forward(self, keep: bool = True):
        """Run the T steps; with keep=False no checkpoint is stored (no reverse).
        One library call per segment (rlb_advance_g)."""
        sv = self.sv
        s0 = sv.g_state().clone()
        tmp = sv.new_g()
        if not keep:
            self.ckpt = []
            self.final = sv.new_g()
            sv.advance_g(s0, self.final, tmp, self.T)
            return sv.fields_g(self.final)
        # each segment advances straight into the next checkpoint's buffer
        self.ckpt = [s0]
        cur = s0
        for k in range(self.K):
            n = min(self.S, self.T - k * self.S)
            nxt = sv.new_g()
            sv.advance_g(cur, nxt, tmp, max(n, 0))
            if k + 1 < self.K:
                self.ckpt.append(nxt)
            cur = nxt
        self.final = cur
        return sv.fields_g(self.final)

    def backward(self, dLde: torch.Tensor, dLdb: torch.Tensor):
        """Reverse sweep, one rlb_trajectory_g + one rlb_adjoint_sweep per
        segment; the parameter partials stay pending across segments and are
        reduced once, so the result does not depend on the segment length."""
        sv = self.sv
        dev = sv.device
        dtau = torch.zeros(sv.batch, dtype=torch.float64, device=dev)
        dbin = torch.zeros(3, dtype=torch.float64, device=dev)
        dein = torch.zeros(1, dtype=torch.float64, device=dev)
        self._lam = [sv.new_lam(), sv.new_lam()]
        self._reader = False  # form of lambda in self._lam[0]
        sv.moments_adjoint(self.final, dLde.contiguous(), dLdb.contiguous(), self._lam[0])
        # the innermost segment's states after its first (which is the
        # checkpoint itself, read in place)
        self._seq = sv.new_g_seq(max(1, min(self.lens[-1], max(self.T, 1)) - 1))
        # per inner level: a ping-pong buffer and its checkpoint buffers
        self._inner = []
        for lv in range(1, len(self.lens)):
            kmax = (self.lens[lv - 1] + self.lens[lv] - 1) // self.lens[lv]
            self._inner.append((sv.new_g(), [sv.new_g() for _ in range(kmax - 1)]))
        if self._overlap():
            self._reverse_overlapped()
        else:
            for k in range(self.K - 1, -1, -1):
                n = min(self.S, self.T - k * self.S)
                if n > 0:
                    self._reverse(self.ckpt[k], n, 1)
        la = self._lam[0]
        if self._reader:
            sv.lam_gather(la, self._lam[1])
            la = self._lam[1]
        self._seq = self._inner = None
        sv.adjoint_flush(dtau, dbin, dein)
        dtc = None
        if sv.tau_cell is not None:
            dtc = torch.zeros(sv.cells, dtype=torch.float64, device=dev)
            sv.adjoint_flush_tau_field(dtc)
        de0 = torch.empty(sv.cells, dtype=torch.float64, device=dev)
        db0 = torch.empty((3, sv.cells), dtype=torch.float64, device=dev)
        sv.init_adjoint(la, de0, db0, dbin, dein)
        self._lam = None
        return dtau, dein, dbin, de0, db0, dtc

    def _overlap(self) -> bool:
        return (OVERLAP_RECOMPUTE and len(self.lens) == 1 and self.K > 1 and self.S > 1
                and self.sv.cells <= OVERLAP_MAX_CELLS and str(self.sv.device).startswith("cuda"))

    def _reverse_overlapped(self):
        """The sqrt(T) reverse pass with each segment's recompute overlapped with
        the previous segment's adjoint sweep: a second solver of the same
        problem on its own stream (default priority) recomputes segment k-1
        into one of two sequence buffers while segment k is swept from the
        other; events order the buffer reuse.  Small lattices leave most of
        the device idle in each launch, so the two run side by side.  The
        kernels and their order per buffer are those of the plain pass, so
        the gradient is the same bit for bit."""
        sv = self.sv
        rc = self._helper()
        s1, s2 = sv.stream, rc.stream
        s2.wait_stream(s1)  # checkpoints and lambda_T are ready
        seqs = [self._seq, sv.new_g_seq(self._seq.shape[0])]
        seqs[1].record_stream(s2)
        self._seq.record_stream(s2)
        ready, free = {}, [None, None]

        def recompute(k):
            n = min(self.S, self.T - k * self.S)
            buf = seqs[k % 2]
            if free[k % 2] is not None:
                s2.wait_event(free[k % 2])
            if n > 1:
                rc.step_g(self.ckpt[k], buf[0])
                rc.trajectory_g(buf, n - 1)
            ev = torch.cuda.Event()
            ev.record(s2)
            ready[k] = ev

        recompute(self.K - 1)
        for k in range(self.K - 1, -1, -1):
            if k > 0:
                recompute(k - 1)
            s1.wait_event(ready.pop(k))
            n = min(self.S, self.T - k * self.S)
            self._segment(self.ckpt[k], seqs[k % 2], n)
            ev = torch.cuda.Event()
            ev.record(s1)
            free[k % 2] = ev

    def _segment(self, start: torch.Tensor, seq: torch.Tensor, n: int):
        """The n reverse steps of the states (start, seq[0], ..., seq[n-2]) in
        one library call, lambda kept in reader form."""
        la, lb = self._lam
        res = self.sv.adjoint_segment(start, seq if n > 1 else None, n, la, lb,
                                      in_reader=self._reader, out_reader=True)
        self._lam = [res, lb if res is la else la]
        self._reader = True

    def _helper(self) -> Solver:
        """The recompute solver of _reverse_overlapped (built once per run)."""
        if getattr(self, "_rc", None) is None:
            sv = self.sv
            self._rc = Solver(sv.setup, device=str(sv.device),
                              stream=torch.cuda.Stream(device=sv.device))
            if sv.tau_cell is not None:
                self._rc.set_tau_field(sv.tau_cell)
        return self._rc

    def close(self):
        if getattr(self, "_rc", None) is not None:
            self._rc.close()
            self._rc = None

    def _reverse(self, start: torch.Tensor, n: int, lv: int):
        """Adjoint steps down through the n steps that begin at state `start`
        (lambda at their end in self._lam[0] on entry, at their beginning on
        return).  Level lv splits them into sub-segments of self.lens[lv]
        steps, recomputing the sub-segment checkpoints from `start`; past the
        innermost level the n states are recomputed and swept."""
        sv = self.sv
        if lv >= len(self.lens):
            # states start+1 .. start+n-1 into the sequence buffer, then the n
            # reverse steps down to `start`, read in place
            seq = self._seq
            if n > 1:
                sv.step_g(start, seq[0])
                sv.trajectory_g(seq, n - 1)
            self._segment(start, seq, n)
            return
        L = self.lens[lv]
        tmp, bufs = self._inner[lv - 1]
        m = (n + L - 1) // L
        cks = [start]
        for j in range(1, m):
            sv.advance_g(cks[-1], bufs[j - 1], tmp, L)
            cks.append(bufs[j - 1])
        for j in range(m - 1, -1, -1):
            self._reverse(cks[j], min(L, n - j * L), lv + 1)


class RLBFunction(torch.autograd.Function):
    """(tau[batch], e_in[1], beta_in[3], e0[cells], beta0[3, cells], tau_cell[cells] or None)
    -> (e_T, beta_T).

    ``setup`` fixes everything else (extents, boundaries, storage, n0, solid);
    ``steps`` is T and ``checkpoint`` is "sqrt", "3level", "store_all" or a
    segment length.
    With ``tau_cell`` the per-cell relaxation times replace tau (whose gradient
    is then the one for a uniform shift of each instance's field).  Inputs may
    live on any device; the run uses ``setup``'s GPU (cuda:0).
    """

    @staticmethod
    def forward(ctx, tau, e_in, beta_in, e0, beta0, tau_cell, setup, steps, checkpoint="sqrt"):
        if getattr(setup, "eta_s", 0.0) > 0.0:
            raise ValueError("the reverse sweep needs a state-independent tau (eta/s not held)")
        tau_h = tau.detach().double().cpu().numpy()
        inflow = list(setup.inflow)
        inflow[1] = float(e_in.detach().double().reshape(-1)[0])
        inflow[2:5] = [float(v) for v in beta_in.detach().double().reshape(-1).cpu()]
        s = replace(setup, tau=tau_h, inflow=tuple(inflow),
                    e0=e0.detach().double().cpu().numpy().reshape(-1),
                    beta0=beta0.detach().double().cpu().numpy().reshape(3, -1), tau_cell=None)
        sv = Solver(s)
        if tau_cell is not None:
            sv.set_tau_field(tau_cell.detach())
        run = GRun(sv, int(steps), schedule(int(steps), checkpoint))
        need = any(ctx.needs_input_grad[:6])
        e, b = run.forward(keep=need)
        if not need:
            sv.close()
            run = None
        ctx.run = run
        ctx.has_tc = tau_cell is not None
        ctx.devs = (tau.device, e_in.device, beta_in.device, e0.device, beta0.device,
                    tau_cell.device if tau_cell is not None else None)
        ctx.shapes = (tau.shape, e_in.shape, beta_in.shape, e0.shape, beta0.shape,
                      tau_cell.shape if tau_cell is not None else None)
        return e.to(e0.device), b.to(beta0.device)

    @staticmethod
    def backward(ctx, g_e, g_b):
        run = ctx.run
        dev = run.sv.device
        if g_e is None:
            g_e = torch.zeros(run.sv.cells, dtype=torch.float64, device=dev)
        if g_b is None:
            g_b = torch.zeros((3, run.sv.cells), dtype=torch.float64, device=dev)
        dtau, dein, dbin, de0, db0, dtc = run.backward(g_e.to(dev, torch.float64),
                                                       g_b.to(dev, torch.float64))
        outs = []
        for g, d, sh in zip((dtau, dein, dbin, de0, db0, dtc), ctx.devs, ctx.shapes):
            outs.append(None if g is None else g.to(d).reshape(sh))
        run.close()
        run.sv.close()
        ctx.run = None
        return (*outs, None, None, None)


def rlb_run(setup, steps: int, tau=None, e_in=None, beta_in=None, e0=None, beta0=None,
            checkpoint="sqrt", device="cuda:0", tau_cell=None):
    """Differentiable run: returns (e_T, beta_T) device float64 tensors.  Any
    parameter left None is taken from ``setup`` as a constant (tau_cell:
    ``setup.tau_cell`` if set, else the per-instance tau)."""
    f64 = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device=device)
    tau = f64(np.asarray(setup.tau).reshape(-1)) if tau is None else tau
    e_in = f64([setup.inflow[1]]) if e_in is None else e_in
    beta_in = f64(setup.inflow[2:5]) if beta_in is None else beta_in
    e0 = f64(np.asarray(setup.e0).reshape(-1)) if e0 is None else e0
    beta0 = f64(np.asarray(setup.beta0).reshape(3, -1)) if beta0 is None else beta0
    if tau_cell is None and getattr(setup, "tau_cell", None) is not None:
        tau_cell = f64(np.asarray(setup.tau_cell).reshape(-1))
    return RLBFunction.apply(tau, e_in, beta_in, e0, beta0, tau_cell, setup, steps, checkpoint)


def surface_mask(setup) -> np.ndarray:
    """Fluid cells with at least one solid D3Q19 neighbour (wrapping across
    periodic faces; nothing lies beyond a non-periodic face)."""
    if setup.solid is None:
        return np.zeros(setup.cells, dtype=bool)
    sol = setup.solid.reshape(setup.batch, setup.nz, setup.ny, setup.nx).astype(bool)
    near = np.zeros_like(sol)
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if 0 < dx * dx + dy * dy + dz * dz <= 2]
    for dx, dy, dz in offs:
        # sh[b, z, y, x] = sol[b, z + dz, y + dy, x + dx]
        sh = np.roll(sol, shift=(-dz, -dy, -dx), axis=(1, 2, 3))
        for axis, d, n, bci in ((3, dx, setup.nx, 0), (2, dy, setup.ny, 1), (1, dz, setup.nz, 2)):
            if d != 0 and setup.bc[bci][0] != 0:
                idx = [slice(None)] * 4
                idx[axis] = n - 1 if d > 0 else 0
                sh[tuple(idx)] = False
        near |= sh
    return (near & ~sol).reshape(-1)
