"""Index rules of in-place (AA-pattern) streaming, checked on the CPU.

A model of the two in-place kernels' reads and writes (the pull kernel: pull
from the swapped layout, push each post-collision value to every cell that
will pull it, clamped pulls through per-face copies; the local kernel: collide
in place, store into the opposite slot, refresh the face copies of the
directions a clamped pull reads) is run on
unique labels with the collision replaced by the identity, so that only data
movement remains.  Checked:

  * within each kernel every location of the state buffer is read by at most
    one cell and written by at most one cell, and by the same cell when both
    (the kernels are race-free in place);
  * the labels after a pull kernel and a local kernel equal those after two
    steps of two-buffer pull streaming (wrap, clamp, bounce-back off solids,
    inflow cells held), and the pull kernel's output holds exactly the values
    the next step pulls.

The reference is the two-buffer streaming rule of the scheme (pull from
x - e_q, resolved per axis, bounce-back off a solid resolved source).
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
        self.inflow_faces = [(a, side) for a in range(3) for side in range(2)
                             if s.bc[a][side] == ri.INFLOW]
        self.solid = np.zeros(s.cells, bool) if s.solid is None else s.solid.astype(bool)
        self.cells = s.cells
        # faces of non-periodic axes, flattened in (axis, side) order
        self.face_id = {}
        self.face_start = []
        acc = 0
        for a in range(3):
            if self.per[a]:
                continue
            u, v = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
            for side in range(2):
                self.face_id[(a, side)] = len(self.face_start)
                self.face_start.append(acc)
                acc += self.n[u] * self.n[v]
        self.nf = acc

    def idx(self, c):
        return (c[2] * self.n[1] + c[1]) * self.n[0] + c[0]

    def coord(self, i):
        return (i % self.n[0], (i // self.n[0]) % self.n[1], i // (self.n[0] * self.n[1]))

    def resolve(self, a, r):
        n = self.n[a]
        if self.per[a]:
            return r % n
        return min(max(r, 0), n - 1)

    def is_inflow(self, c):
        return any(c[a] == (0 if side == 0 else self.n[a] - 1) for a, side in self.inflow_faces)

    def solid_at(self, c):
        return bool(self.solid[self.idx(c)])

    def near(self, c):
        for q in range(1, Q):
            src = tuple(self.resolve(a, c[a] - E[q][a]) for a in range(3))
            if self.solid_at(src):
                return True
        return False

    def plain(self, c):
        """Fast path of the pull kernel: no solid neighbour, not inflow, off
        every face of a non-periodic axis."""
        if self.solid_at(c) or self.near(c) or self.is_inflow(c):
            return False
        return all(self.per[a] or 1 <= c[a] <= self.n[a] - 2 for a in range(3))

    def face_pos(self, f, a, c):
        u, v = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
        return self.face_start[f] + c[v] * self.n[u] + c[u]

    def faces_of(self, c):
        for a in range(3):
            if self.per[a]:
                continue
            if c[a] == 0:
                yield a, 0
            elif c[a] == self.n[a] - 1:
                yield a, 1


class Access:
    """Reads and writes of one kernel, per location, by cell."""

    def __init__(self):
        self.readers, self.writers = {}, {}

    def read(self, store, key, cell):
        self.readers.setdefault((store, key), set()).add(cell)

    def write(self, store, key, cell):
        self.writers.setdefault((store, key), set()).add(cell)

    def check(self):
        """State buffer: one reader and one writer per location, the same cell.
        Face copies: written by one cell at most, and never in a kernel that
        reads them (several clamped readers may share a copy)."""
        for loc, who in self.readers.items():
            if loc[0] == "A":
                assert len(who) == 1, ("read by several cells", loc, who)
        for loc, who in self.writers.items():
            assert len(who) == 1, ("written by several cells", loc, who)
            if loc in self.readers:
                assert loc[0] == "A" and who == self.readers[loc], \
                    ("read and written by different cells", loc)


def reference_step(L: Lat, S, held):
    """Two-buffer pull streaming with identity collision: S[q][cell] labels."""
    out = np.empty_like(S)
    for i in range(L.cells):
        c = L.coord(i)
        if L.solid[i]:
            out[:, i] = -1
            continue
        if L.is_inflow(c):
            out[:, i] = held
            continue
        for q in range(Q):
            src = tuple(L.resolve(a, c[a] - E[q][a]) for a in range(3))
            out[q, i] = S[OPP[q], i] if L.solid_at(src) else S[q, L.idx(src)]
    return out


def local_kernel(L: Lat, A, Fb, held, acc: Access):
    """Streamed -> swapped: collide in place (identity), store into the
    opposite slot; face cells refresh their face copies."""
    newA = A.copy()
    newF = Fb.copy()
    for i in range(L.cells):
        c = L.coord(i)
        if L.solid[i]:
            continue
        pre = []
        for q in range(Q):
            acc.read("A", (q, i), i)
            pre.append(A[q, i])
        post = list(held) if L.is_inflow(c) else pre
        for q in range(Q):
            acc.write("A", (OPP[q], i), i)
            newA[OPP[q], i] = post[q]
        if L.nf and not L.plain(c):
            for a, side in L.faces_of(c):
                t = L.face_pos(L.face_id[(a, side)], a, c)
                for q in range(Q):
                    # only the directions a clamped pull onto this face reads
                    if E[q][a] != (1 if side == 0 else -1):
                        continue
                    acc.write("F", (q, t), i)
                    newF[q, t] = post[q]
    return newA, newF


def pull_kernel(L: Lat, A, Fb, held, acc: Access):
    """Swapped -> streamed: pull (plain: slot opp(q) of the source; bounce:
    slot q of the cell; clamped: the face copy of the first clamped axis),
    collide (identity), push S(x)_q to slot q of every cell that will pull
    it."""
    newA = A.copy()
    for i in range(L.cells):
        c = L.coord(i)
        if L.solid[i]:
            continue
        inflow = L.is_inflow(c)
        pre = [None] * Q
        if inflow:
            pre = list(held)
        else:
            for q in range(Q):
                src = tuple(L.resolve(a, c[a] - E[q][a]) for a in range(3))
                bounce = L.solid_at(src)
                clamp_axis = None
                for a in (2, 1, 0):
                    r = c[a] - E[q][a]
                    if not L.per[a] and (r < 0 or r >= L.n[a]):
                        clamp_axis = (a, 0 if r < 0 else 1)
                if clamp_axis is not None and not bounce:
                    a, side = clamp_axis
                    t = L.face_pos(L.face_id[(a, side)], a, src)
                    acc.read("F", (q, t), i)
                    pre[q] = Fb[q, t]
                elif bounce:
                    acc.read("A", (q, i), i)
                    pre[q] = A[q, i]
                else:
                    acc.read("A", (OPP[q], L.idx(src)), i)
                    pre[q] = A[OPP[q], L.idx(src)]
        post = pre
        for q in range(Q):
            e = E[q]
            # readers whose pull of q resolves to this cell, per clamp pattern m
            for m in range(8):
                if any((m >> d) & 1 and e[d] == 0 for d in range(3)):
                    continue
                ok = True
                rc = [0, 0, 0]
                off = [0, 0, 0]
                for d in range(3):
                    n = L.n[d]
                    if (m >> d) & 1:
                        ok = ok and not L.per[d] and ((e[d] == 1 and c[d] == 0) or
                                                      (e[d] == -1 and c[d] == n - 1))
                        rc[d] = c[d]
                    else:
                        r = c[d] + e[d]
                        if L.per[d]:
                            r %= n
                        else:
                            ok = ok and 0 <= r < n
                        rc[d] = r
                        off[d] = e[d]
                if not ok:
                    continue
                offc = tuple(L.resolve(d, c[d] + off[d]) for d in range(3))
                if L.solid_at(offc) or L.is_inflow(tuple(rc)):
                    continue
                j = L.idx(tuple(rc))
                acc.write("A", (q, j), i)
                newA[q, j] = post[q]
            # bounce-back receiver: this cell, when its pull of opp(q) hits a solid
            if not inflow:
                tgt = tuple(L.resolve(d, c[d] + e[d]) for d in range(3))
                if L.solid_at(tgt):
                    acc.write("A", (OPP[q], i), i)
                    newA[OPP[q], i] = post[q]
    return newA


CASES = {
    "periodic": lambda: ri.random_state_setup(5, 4, 6, seed=1),
    "outflow_all": lambda: ri.random_state_setup(4, 5, 6, seed=2, bc=((ri.OUTFLOW, ri.OUTFLOW),) * 3),
    "inflow_obstacle": lambda: ri.random_state_setup(
        9, 6, 7, seed=3, bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC),
                             (ri.OUTFLOW, ri.OUTFLOW)),
        solid_centre=(4, 3, 3), solid_radius=1.7),
    "solid_on_face": lambda: ri.random_state_setup(
        7, 6, 5, seed=4, bc=((ri.OUTFLOW, ri.INFLOW), (ri.OUTFLOW, ri.OUTFLOW),
                             (ri.PERIODIC, ri.PERIODIC)),
        solid_centre=(0, 3, 2), solid_radius=1.5),
    "thin_and_one_cell_axes": lambda: ri.random_state_setup(
        2, 1, 5, seed=5, bc=((ri.OUTFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC),
                             (ri.OUTFLOW, ri.INFLOW))),
}


@pytest.mark.parametrize("name", list(CASES))
def test_inplace_kernels_race_free_and_equal_two_buffer_streaming(name):
    s = CASES[name]()
    L = Lat(s)
    rng = np.random.default_rng(0)
    S0 = rng.permutation(Q * L.cells).reshape(Q, L.cells).astype(np.int64) + 1000
    held = np.arange(Q, dtype=np.int64) + 10
    for i in range(L.cells):
        if L.solid[i]:
            S0[:, i] = -1
        elif L.is_inflow(L.coord(i)):
            S0[:, i] = held
    # initial swapped layout and face copies (the in-place set-up)
    A = np.full((Q, L.cells), -7, dtype=np.int64)
    Fb = np.full((Q, max(L.nf, 1)), -9, dtype=np.int64)
    for i in range(L.cells):
        if L.solid[i]:
            continue
        for q in range(Q):
            A[OPP[q], i] = S0[q, i]
        for a, side in L.faces_of(L.coord(i)):
            Fb[:, L.face_pos(L.face_id[(a, side)], a, L.coord(i))] = S0[:, i]
    ref = S0
    for _ in range(3):  # three pull + local pairs
        acc = Access()
        A = pull_kernel(L, A, Fb, held, acc)
        acc.check()
        ref1 = reference_step(L, ref, held)
        # streamed layout: slot q of x holds what x pulls at the next step
        nxt = reference_step(L, ref1, held)
        for i in range(L.cells):
            c = L.coord(i)
            if L.solid[i] or L.is_inflow(c):
                continue
            assert list(A[:, i]) == list(nxt[:, i]), (name, i)
        acc = Access()
        A, Fb = local_kernel(L, A, Fb, held, acc)
        acc.check()
        ref = nxt
        for i in range(L.cells):
            if L.solid[i]:
                continue
            assert [A[OPP[q], i] for q in range(Q)] == list(ref[:, i]), (name, i)
