"""Python face of librlb.so: device buffers and streams from PyTorch, all
arithmetic in the library's HIP kernels (argument marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import check

STORAGE_DTYPE = {
    _lib.F64: torch.float64,
    _lib.F32: torch.float32,
    _lib.F32DEV: torch.float32,
    _lib.F16DEV: torch.float16,
    _lib.BF16DEV: torch.bfloat16,
}
Q = 19
BRICK = 64  # cells per brick of the population layout


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_params(nx, ny, nz, batch=1, c_l=1.0, bc=((0, 0), (0, 0), (0, 0)),
                inflow=(1.0, 1.0, 0.0, 0.0, 0.0), storage=_lib.F64, n_ref=1.0,
                e_ref=1.0, collide=_lib.COLLIDE_AUTO, kappa=0.0, inplace=False) -> _lib.Params:
    p = _lib.Params()
    p.nx, p.ny, p.nz, p.batch = int(nx), int(ny), int(nz), int(batch)
    p.c_l = float(c_l)
    for a in range(3):
        for s in range(2):
            p.bc[a][s] = int(bc[a][s])
    p.inflow_n, p.inflow_e = float(inflow[0]), float(inflow[1])
    for k in range(3):
        p.inflow_beta[k] = float(inflow[2 + k])
    p.storage = int(storage)
    p.n_ref, p.e_ref = float(n_ref), float(e_ref)
    p.collide = int(collide)
    p.kappa = float(kappa)
    p.inplace = 1 if inplace else 0
    return p


def _lattice_tables():
    """(e[19][3], w[19], opp[19]) of the D3Q19 ordering the library uses
    (0 rest; +x,-x,+y,-y,+z,-z; then the xy, xz, yz diagonal pairs)."""
    e = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
         (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    opp = [e.index(tuple(-v for v in d)) for d in e]
    w = [1 / 3 if sum(map(abs, d)) == 0 else (1 / 18 if sum(map(abs, d)) == 1 else 1 / 36) for d in e]
    return e, w, opp


def unpack_block(t: torch.Tensor, cells: int) -> torch.Tensor:
    """Population block(s) [..., bricks, 19, 64] -> [..., 19, cells] (a copy)."""
    lead = t.shape[:-3]
    u = t.movedim(-2, -3).reshape(*lead, Q, t.shape[-3] * BRICK)
    return u[..., :cells].clone()


def pack_block(a, nbrick: int, cells: int, dtype, device, fill: float = 0.0) -> torch.Tensor:
    """[..., 19, cells] -> population block(s) [..., bricks, 19, 64] (element
    (q, cell) at (cell // 64) * 19 * 64 + q * 64 + cell % 64); padding = fill."""
    a = torch.as_tensor(a)
    lead = a.shape[:-2]
    full = torch.full((*lead, Q, nbrick * BRICK), fill, dtype=dtype, device=device)
    full[..., :cells] = a.to(device, dtype)
    return full.reshape(*lead, Q, nbrick, BRICK).movedim(-3, -2).contiguous()


def buffer_layout(p: _lib.Params) -> Tuple[int, int]:
    qs = ctypes.c_int64()
    nb = ctypes.c_int64()
    check(_lib.lib().rlb_buffer_layout(ctypes.byref(p), ctypes.byref(qs), ctypes.byref(nb)),
          "rlb_buffer_layout")
    return qs.value, nb.value


class Solver:
    """One RLB lattice problem resident on a GPU.

    ``setup`` is any object with the attributes of ``rlb_inputs.Setup`` (extents,
    batch, c_l, bc, inflow, tau, storage, n_ref, e_ref, n0, e0, beta0, solid).
    """

    def __init__(self, setup, device: str = "cuda:0", stream: Optional[torch.cuda.Stream] = None):
        _lib.lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        s = setup
        self.setup = s
        self.params = make_params(s.nx, s.ny, s.nz, s.batch, s.c_l, s.bc, s.inflow, s.storage,
                                  s.n_ref, s.e_ref, getattr(s, "collide", _lib.COLLIDE_AUTO),
                                  getattr(s, "kappa", 0.0), getattr(s, "inplace", False))
        self.inplace = bool(getattr(s, "inplace", False))
        self.nx, self.ny, self.nz, self.batch = s.nx, s.ny, s.nz, s.batch
        self.cells = s.batch * s.nz * s.ny * s.nx
        self.storage = int(s.storage)
        self.dtype = STORAGE_DTYPE[self.storage]
        self.lam_dtype = torch.float64  # adjoint buffers are FP64 for every storage
        self.q_stride, self.state_bytes = buffer_layout(self.params)
        self.nbrick = self.q_stride // BRICK
        with torch.cuda.stream(self.stream):
            self.pop = [torch.empty((2, self.nbrick, Q, BRICK), dtype=self.dtype,
                                    device=self.device) for _ in range(1 if self.inplace else 2)]
            f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
            n0 = f64(np.asarray(s.n0).reshape(-1))
            e0 = f64(np.asarray(s.e0).reshape(-1))
            b0 = f64(np.asarray(s.beta0).reshape(3, -1))
            self.e0_dev, self.beta0_dev = e0, b0
            self.solid = None
            if s.solid is not None:
                self.solid = torch.as_tensor(np.ascontiguousarray(s.solid.reshape(-1), np.uint8)).to(self.device)
        self.tau = np.ascontiguousarray(np.asarray(s.tau, dtype=np.float64).reshape(-1))
        if self.tau.size == 1 and self.batch > 1:
            self.tau = np.full(self.batch, self.tau[0])
        h = ctypes.c_void_p()
        check(_lib.lib().rlb_init(ctypes.byref(h), ctypes.byref(self.params),
                                  self.tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _ptr(self.solid), _ptr(n0), _ptr(e0), _ptr(b0),
                                  _ptr(self.pop[0]), _ptr(self.pop[-1]) if not self.inplace else None,
                                  ctypes.c_void_p(self.stream.cuda_stream)), "rlb_init")
        self.h = h
        self.tau_cell = None
        if getattr(s, "tau_cell", None) is not None:
            self.set_tau_field(s.tau_cell)
        if getattr(s, "eta_s", 0.0) > 0.0:
            self.hold_eta_over_s(s.eta_s, getattr(s, "d_G", 16.0))

    # ------------------------------------------------------------------ forward
    def step(self, nsteps: int = 1):
        check(_lib.lib().rlb_step(self.h, int(nsteps)), "rlb_step")

    def step_g(self, g_src: torch.Tensor, g_dst: torch.Tensor):
        check(_lib.lib().rlb_step_g(self.h, _ptr(g_src), _ptr(g_dst)), "rlb_step_g")

    def advance_g(self, g_src: torch.Tensor, g_dst: torch.Tensor, g_tmp: torch.Tensor, n: int):
        """n g-only steps from g_src into g_dst (g_tmp: ping-pong buffer)."""
        check(_lib.lib().rlb_advance_g(self.h, _ptr(g_src), _ptr(g_dst), _ptr(g_tmp), int(n)),
              "rlb_advance_g")

    def new_g_seq(self, n: int) -> torch.Tensor:
        """n contiguous g blocks, [n][bricks][19][64]."""
        return torch.empty((n, self.nbrick, Q, BRICK), dtype=self.dtype, device=self.device)

    def _seq_stride(self, g_seq: torch.Tensor) -> int:
        if g_seq.dim() != 4 or tuple(g_seq.shape[1:]) != (self.nbrick, Q, BRICK) \
                or not g_seq.is_contiguous():
            raise ValueError("g_seq must be a contiguous [n][bricks][19][64] tensor")
        if g_seq.dtype != self.dtype:
            raise ValueError("g_seq dtype does not match the storage format")
        return Q * self.q_stride * g_seq.element_size()

    def trajectory_g(self, g_seq: torch.Tensor, n: int):
        """Blocks 1 .. n-1 of g_seq recomputed from block 0."""
        if not 1 <= n <= g_seq.shape[0]:
            raise ValueError("n out of range for g_seq")
        check(_lib.lib().rlb_trajectory_g(self.h, _ptr(g_seq), self._seq_stride(g_seq), int(n)),
              "rlb_trajectory_g")

    def adjoint_sweep(self, g_seq: torch.Tensor, n: int, lam_a: torch.Tensor,
                      lam_b: torch.Tensor) -> torch.Tensor:
        """n reverse steps over blocks n-1 .. 0 of g_seq, starting from lam_a;
        returns the buffer (lam_a or lam_b) holding the result.  Parameter
        contributions stay pending until adjoint_flush."""
        if not 0 <= n <= g_seq.shape[0]:
            raise ValueError("n out of range for g_seq")
        res = ctypes.c_void_p()
        check(_lib.lib().rlb_adjoint_sweep(self.h, _ptr(g_seq), self._seq_stride(g_seq), int(n),
                                           _ptr(lam_a), _ptr(lam_b), ctypes.byref(res)),
              "rlb_adjoint_sweep")
        return lam_a if res.value == lam_a.data_ptr() else lam_b

    def adjoint_segment(self, g_first: Optional[torch.Tensor], g_seq: Optional[torch.Tensor],
                        n: int, lam_a: torch.Tensor, lam_b: torch.Tensor,
                        in_reader: bool = False, out_reader: bool = False) -> torch.Tensor:
        """n reverse steps over the states (g_first, g_seq[0], ..., g_seq[n-2])
        (or g_seq[0 .. n-1] without g_first), lambda in lam_a in reader or
        natural form; returns the buffer (lam_a or lam_b) holding the result
        (reader form with out_reader)."""
        blocks = n - 1 if g_first is not None else n
        if g_seq is not None:
            if not 0 <= blocks <= g_seq.shape[0]:
                raise ValueError("n out of range for g_seq")
            stride = self._seq_stride(g_seq)
        elif blocks > 0:
            raise ValueError("g_seq is needed for n > 1")
        else:
            stride = 0
        flags = (_lib.LAM_IN_READER if in_reader else 0) | (_lib.LAM_OUT_READER if out_reader else 0)
        res = ctypes.c_void_p()
        check(_lib.lib().rlb_adjoint_segment(self.h, _ptr(g_first), _ptr(g_seq), int(stride), int(n),
                                             _ptr(lam_a), _ptr(lam_b), int(flags),
                                             ctypes.byref(res)), "rlb_adjoint_segment")
        return lam_a if res.value == lam_a.data_ptr() else lam_b

    def lam_gather(self, lam_reader: torch.Tensor, lam_out: torch.Tensor):
        """Natural lambda from its reader form."""
        check(_lib.lib().rlb_lam_gather(self.h, _ptr(lam_reader), _ptr(lam_out)), "rlb_lam_gather")

    def adjoint_flush(self, dtau=None, dbeta_in=None, de_in=None):
        check(_lib.lib().rlb_adjoint_flush(self.h, _ptr(dtau), _ptr(dbeta_in), _ptr(de_in)),
              "rlb_adjoint_flush")

    # ------------------------------------------------------------- relaxation
    def set_tau_field(self, tau_cell):
        """Per-cell relaxation times (array/tensor [cells]) or None for the
        per-instance tau."""
        if tau_cell is None:
            check(_lib.lib().rlb_set_tau_field(self.h, None), "rlb_set_tau_field")
            self.tau_cell = None
            return
        t = torch.as_tensor(np.asarray(tau_cell, dtype=np.float64).reshape(-1)
                            if not isinstance(tau_cell, torch.Tensor) else tau_cell)
        t = t.to(self.device, torch.float64).reshape(-1).contiguous()
        if t.numel() != self.cells:
            raise ValueError("tau field must have one value per cell")
        check(_lib.lib().rlb_set_tau_field(self.h, _ptr(t)), "rlb_set_tau_field")
        self.tau_cell = t

    def hold_eta_over_s(self, eta_over_s: float, d_G: float = 16.0):
        check(_lib.lib().rlb_hold_eta_over_s(self.h, float(eta_over_s), float(d_G)),
              "rlb_hold_eta_over_s")

    def transport(self, d_G: float = 16.0):
        """(T, s, eta, eta/s) device float64 [cells] of the current state."""
        out = [torch.empty(self.cells, dtype=torch.float64, device=self.device) for _ in range(4)]
        check(_lib.lib().rlb_transport(self.h, float(d_G), *[_ptr(o) for o in out]),
              "rlb_transport")
        return tuple(out)

    def adjoint_flush_tau_field(self, out: torch.Tensor):
        check(_lib.lib().rlb_adjoint_flush_tau_field(self.h, _ptr(out)),
              "rlb_adjoint_flush_tau_field")

    def state(self) -> torch.Tensor:
        """The buffer holding the current state, [2][bricks][19][64] (the buffer itself,
        not a copy; see unpack)."""
        p = ctypes.c_void_p()
        check(_lib.lib().rlb_current(self.h, ctypes.byref(p)), "rlb_current")
        for t in self.pop:
            if t.data_ptr() == p.value:
                return t
        raise RuntimeError("current state is not one of the solver's buffers")

    def populations(self) -> torch.Tensor:
        """The current stored state S_t as [2][19][cells] in the natural slot
        order (a copy; the in-place layout is un-swapped)."""
        st = self.unpack(self.state())
        if self.inplace:
            _, _, opp = _lattice_tables()
            st = st[:, opp]
        return st

    def g_state(self) -> torch.Tensor:
        return self.state()[1]

    def new_g(self) -> torch.Tensor:
        """A g block, [bricks][19][64] in the storage format."""
        return torch.empty((self.nbrick, Q, BRICK), dtype=self.dtype, device=self.device)

    def new_lam(self) -> torch.Tensor:
        """An adjoint buffer, [bricks][19][64] float64."""
        return torch.empty((self.nbrick, Q, BRICK), dtype=self.lam_dtype, device=self.device)

    # Layout conversion for host-side inspection and test I/O (no arithmetic):
    # a population block stores bricks of 64 cells with their 19 directions
    # one after another; unpack gives the plain [19][cells] view of the values.
    def unpack(self, t: torch.Tensor) -> torch.Tensor:
        """[..., bricks, 19, 64] -> [..., 19, cells] (a copy)."""
        return unpack_block(t, self.cells)

    def pack(self, a, dtype=None, fill: float = 0.0) -> torch.Tensor:
        """[..., 19, cells] (array or tensor) -> [..., bricks, 19, 64]; padding
        cells hold ``fill``."""
        return pack_block(a, self.nbrick, self.cells, self.dtype if dtype is None else dtype,
                          self.device, fill)

    def moments(self, sums: bool = False):
        """(n, e, beta[3]) device float64 tensors of shape [cells] / [3, cells];
        with sums=True also the host [batch][5] conservation sums."""
        n = torch.empty(self.cells, dtype=torch.float64, device=self.device)
        e = torch.empty_like(n)
        b = torch.empty((3, self.cells), dtype=torch.float64, device=self.device)
        out = None
        sp = None
        if sums:
            out = np.zeros((self.batch, 5))
            sp = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        check(_lib.lib().rlb_moments(self.h, _ptr(n), _ptr(e), _ptr(b), sp), "rlb_moments")
        return (n, e, b, out) if sums else (n, e, b)

    def moments_noalloc(self, n: torch.Tensor, e: torch.Tensor, beta: torch.Tensor,
                        sums: Optional[torch.Tensor] = None):
        """rlb_moments_noalloc into caller-provided device float64 tensors n, e
        [cells], beta [3, cells] and sums [batch, 5] (or None); asynchronous."""
        check(_lib.lib().rlb_moments_noalloc(self.h, _ptr(n), _ptr(e), _ptr(beta), _ptr(sums)),
              "rlb_moments_noalloc")

    def fields_g(self, g_state: torch.Tensor):
        """(e [cells], beta [3, cells]) device float64 of a g block."""
        e = torch.empty(self.cells, dtype=torch.float64, device=self.device)
        b = torch.empty((3, self.cells), dtype=torch.float64, device=self.device)
        check(_lib.lib().rlb_fields_g(self.h, _ptr(g_state), _ptr(e), _ptr(b)), "rlb_fields_g")
        return e, b

    def counters(self, raise_on_unphysical: bool = False):
        c = (ctypes.c_int64 * 2)()
        st = _lib.lib().rlb_counters(self.h, c)
        if st == _lib.RLB_EUNPHYSICAL and not raise_on_unphysical:
            return int(c[0]), int(c[1])
        check(st, "rlb_counters")
        return int(c[0]), int(c[1])

    # ------------------------------------------------------------------ reverse
    def adjoint_step(self, g_state_t, lam_next, lam_out, dtau=None, dbeta_in=None, de_in=None):
        check(_lib.lib().rlb_adjoint_step(self.h, _ptr(g_state_t), _ptr(lam_next), _ptr(lam_out),
                                          _ptr(dtau), _ptr(dbeta_in), _ptr(de_in)),
              "rlb_adjoint_step")

    def moments_adjoint(self, g_state_T, dLde, dLdb, lam_T):
        check(_lib.lib().rlb_moments_adjoint(self.h, _ptr(g_state_T), _ptr(dLde), _ptr(dLdb),
                                             _ptr(lam_T)), "rlb_moments_adjoint")

    def init_adjoint(self, lam0, de0, db0, dbeta_in=None, de_in=None, e0=None, beta0=None):
        e0 = self.e0_dev if e0 is None else e0
        beta0 = self.beta0_dev if beta0 is None else beta0
        check(_lib.lib().rlb_init_adjoint(self.h, _ptr(e0), _ptr(beta0), _ptr(lam0), _ptr(de0),
                                          _ptr(db0), _ptr(dbeta_in), _ptr(de_in)),
              "rlb_init_adjoint")

    # ------------------------------------------------------------------ misc
    def close(self):
        if getattr(self, "h", None):
            check(_lib.lib().rlb_destroy(self.h), "rlb_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
