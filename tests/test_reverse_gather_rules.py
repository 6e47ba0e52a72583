"""Index rules of the reverse step's reader form, checked on the CPU.

The reverse step stores each update's contributions at its own cell,
R(r)_q = mu_q(r), and the next step gathers lambda from them.  The gather
must equal the transpose of the forward pull map: slot (p, x) of the stored
state receives mu_q(r) from every update r whose pull of direction q read that
slot (the plain reader, a bounce-back off a solid, or a pull clamped onto a
face).  Two models of the kernel's gather rules are checked against the
transpose, built here by running the pull rule itself, on lattices with every
boundary kind, solids next to faces and thin axes:

  * the general rule (any number of non-periodic axes): the plain or
    bounce-back read, then on face cells the readers that lie outside
    dropped and, per clamp pattern, the clamped readers added;
  * the rule for one non-periodic axis A of extent > 1: a cell on A's low
    face adds the reader of each p with e_pA = +1 moved back onto the face
    and drops its reader of opp(p) (unless that pull bounces); a high-face
    cell the mirror image.
"""
import numpy as np
import pytest

import rlb_inputs as ri

E = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
     (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
OPP = [E.index(tuple(-v for v in e)) for e in E]
Q = 19


class Lat:
    def __init__(self, s: ri.Setup):
        self.n = (s.nx, s.ny, s.nz)
        self.per = tuple(s.bc[a][0] == ri.PERIODIC for a in range(3))
        self.inflow = [(a, side) for a in range(3) for side in range(2) if s.bc[a][side] == ri.INFLOW]
        self.cells = s.nx * s.ny * s.nz
        self.solid = np.zeros(self.cells, bool) if s.solid is None else s.solid.astype(bool)

    def idx(self, c):
        return (c[2] * self.n[1] + c[1]) * self.n[0] + c[0]

    def coord(self, i):
        return (i % self.n[0], (i // self.n[0]) % self.n[1], i // (self.n[0] * self.n[1]))

    def resolve(self, a, r):
        n = self.n[a]
        return r % n if self.per[a] else min(max(r, 0), n - 1)

    def src(self, c, q):
        return tuple(self.resolve(a, c[a] - E[q][a]) for a in range(3))

    def held(self, i):
        c = self.coord(i)
        return self.solid[i] or any(c[a] == (0 if side == 0 else self.n[a] - 1)
                                    for a, side in self.inflow)

    def bounce(self, c, q):
        return bool(self.solid[self.idx(self.src(c, q))])


def transpose(L: Lat, R: np.ndarray) -> np.ndarray:
    """lambda[p, x] = sum of R[q, r] over the pulls (r, q) that read slot (p, x)."""
    lam = np.zeros_like(R)
    for r in range(L.cells):
        if L.held(r):
            continue
        c = L.coord(r)
        for q in range(Q):
            if L.bounce(c, q):
                lam[OPP[q], r] += R[q, r]
            else:
                lam[q, L.idx(L.src(c, q))] += R[q, r]
    return lam


def gather_general(L: Lat, R: np.ndarray) -> np.ndarray:
    lam = np.zeros_like(R)
    for x in range(L.cells):
        c = L.coord(x)
        lo = [not L.per[a] and c[a] == 0 for a in range(3)]
        hi = [not L.per[a] and c[a] == L.n[a] - 1 for a in range(3)]
        for p in range(Q):
            q = OPP[p]
            e = E[p]
            if L.bounce(c, q):
                v = R[q, x]
            else:
                v = R[p, L.idx(L.src(c, q))]  # x + e_p, wrapped or clamped
                if any((e[a] == 1 and hi[a]) or (e[a] == -1 and lo[a]) for a in range(3)):
                    v = 0.0  # the plain reader lies outside the domain
            for m in range(1, 8):
                if any((m >> a) & 1 and e[a] == 0 for a in range(3)):
                    continue
                ok, r = True, list(c)
                for a in range(3):
                    if e[a] == 0:
                        continue
                    if (m >> a) & 1:
                        ok = ok and ((e[a] == 1 and lo[a]) or (e[a] == -1 and hi[a]))
                    else:
                        ok = ok and not ((e[a] == 1 and hi[a]) or (e[a] == -1 and lo[a]))
                        r[a] = L.resolve(a, c[a] + e[a])
                if ok:
                    v += R[p, L.idx(tuple(r))]
            lam[p, x] = v
    return lam


def gather_one_axis(L: Lat, R: np.ndarray, A: int) -> np.ndarray:
    lam = np.zeros_like(R)
    for x in range(L.cells):
        c = L.coord(x)
        for p in range(Q):
            q = OPP[p]
            lam[p, x] = R[q, x] if L.bounce(c, q) else R[p, L.idx(L.src(c, q))]
        lo, hi = c[A] == 0, c[A] == L.n[A] - 1
        if not (lo or hi):
            continue
        for p in range(Q):
            if E[p][A] != 1:
                continue
            m = OPP[p]
            # low face: the reader of p, x + e_p moved back onto the face;
            # high face: the reader of m, x + e_m moved forward onto it
            r = list(L.src(c, m) if lo else L.src(c, p))
            r[A] = c[A]
            v = R[p, L.idx(tuple(r))] if lo else R[m, L.idx(tuple(r))]
            bp, bm = L.bounce(c, m), L.bounce(c, p)
            lam[p, x] = lam[p, x] + v if lo else (lam[p, x] if bp else 0.0)
            lam[m, x] = lam[m, x] + v if hi else (lam[m, x] if bm else 0.0)
    return lam


P_, O_, I_ = ri.PERIODIC, ri.OUTFLOW, ri.INFLOW
CASES = {
    "periodic_with_obstacle": dict(n=(6, 5, 4), bc=((P_, P_), (P_, P_), (P_, P_)), ball=((2, 2, 2), 1.2)),
    "x_inflow_outflow_obstacle_on_face": dict(n=(7, 4, 5), bc=((I_, O_), (P_, P_), (P_, P_)),
                                              ball=((6, 2, 2), 1.5)),
    "z_outflow_tube_one_cell_wide": dict(n=(1, 1, 9), bc=((P_, P_), (P_, P_), (O_, O_)), ball=None),
    "y_outflow_two_cells": dict(n=(4, 2, 3), bc=((P_, P_), (O_, O_), (P_, P_)), ball=None),
    "all_outflow_corners": dict(n=(4, 5, 3), bc=((O_, O_), (O_, O_), (O_, O_)), ball=((0, 0, 1), 1.1)),
    "two_thin_outflow_axes": dict(n=(5, 2, 3), bc=((O_, O_), (O_, O_), (I_, O_)), ball=((2, 0, 1), 0.9)),
}


def lattice(name):
    d = CASES[name]
    s = ri.random_state_setup(*d["n"], seed=3, bc=d["bc"], tau=[0.8])
    if d["ball"] is not None:
        s.solid = ri.ball(s, *d["ball"])
    return Lat(s)


@pytest.mark.parametrize("name", list(CASES))
def test_reader_form_gather_is_the_transpose_of_the_pull(name):
    L = lattice(name)
    R = np.random.default_rng(5).standard_normal((Q, L.cells))
    for i in range(L.cells):
        if L.held(i):
            R[:, i] = 0.0  # held cells pull nothing and store zeros
    want = transpose(L, R)
    fluid = ~L.solid  # lambda of solid cells is never used
    assert np.allclose(gather_general(L, R)[:, fluid], want[:, fluid], rtol=0, atol=1e-12)
    axes = [a for a in range(3) if not L.per[a]]
    if len(axes) == 1 and L.n[axes[0]] > 1:
        got = gather_one_axis(L, R, axes[0])
        assert np.allclose(got[:, fluid], want[:, fluid], rtol=0, atol=1e-12)
