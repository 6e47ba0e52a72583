"""Reverse mode on the GPU vs the oracle's reverse mode and finite differences.

Per entry point (rlb_adjoint_step, rlb_moments_adjoint, rlb_init_adjoint) the
GPU result is compared element by element with the oracle's complex-step
transpose of the pull map; the checkpointed reverse sweep is compared with the
oracle's store-all FP64 sweep and with central differences of GPU FP64
forward runs.
"""
import numpy as np
import pytest
import torch

import oracle
import rlb_inputs as ri
from helpers import problem

pytestmark = pytest.mark.gpu


def setups():
    return {
        "periodic_batch": ri.random_state_setup(7, 6, 9, batch=2, seed=201, tau=[0.7, 1.1]),
        "inflow_outflow_obstacle": ri.random_state_setup(
            13, 7, 9, batch=2, seed=202, tau=[0.65, 0.9],
            bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW)),
            inflow=(1.0, 1.05, 0.15, 0.03, -0.02), solid_centre=(6, 3, 4), solid_radius=2.2),
        "outflow_corners": ri.random_state_setup(6, 5, 7, seed=203, tau=[0.8],
                                                 bc=((ri.OUTFLOW, ri.OUTFLOW),) * 3),
        "solid_on_outflow_face": ri.random_state_setup(
            8, 9, 7, seed=204, tau=[0.75],
            bc=((ri.OUTFLOW, ri.INFLOW), (ri.OUTFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC)),
            inflow=(1.0, 0.95, -0.1, 0.05, 0.0), solid_centre=(0, 4, 3), solid_radius=2.0),
        "inflow_x_solid_on_outflow_face": ri.random_state_setup(
            11, 6, 7, batch=2, seed=206, tau=[0.7, 0.95],
            bc=((ri.INFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC), (ri.PERIODIC, ri.PERIODIC)),
            inflow=(1.0, 1.02, 0.12, 0.02, -0.03), solid_centre=(10, 3, 3), solid_radius=1.8),
        "thin_outflow_axis_and_inflow": ri.random_state_setup(
            5, 2, 4, seed=207, tau=[0.85],
            bc=((ri.INFLOW, ri.OUTFLOW), (ri.OUTFLOW, ri.OUTFLOW), (ri.PERIODIC, ri.PERIODIC)),
            inflow=(1.0, 1.0, 0.1, 0.0, 0.02), solid_centre=(3, 1, 2), solid_radius=0.9),
        "tube_batch": ri.shock_tube(nz=67, e_L=1.0, e_R=0.3, tau=0.7, batch=3),
        "tachyon": ri.random_state_setup(6, 7, 5, seed=205, tau=[0.9], c_l=2.0,
                                         bc=((ri.PERIODIC, ri.PERIODIC), (ri.OUTFLOW, ri.OUTFLOW),
                                             (ri.PERIODIC, ri.PERIODIC))),
    }


def upload_g(sv, g: np.ndarray) -> torch.Tensor:
    return sv.pack(g)


def upload_lam(sv, lam: np.ndarray) -> torch.Tensor:
    return sv.pack(lam, dtype=sv.lam_dtype, fill=float("nan"))


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(setups()))
def test_adjoint_step_matches_oracle(name):
    from paper_0912_2913_amd.solver import Solver

    s = setups()[name]
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, 3)
    Sg = np.ascontiguousarray(S[1])
    rng = np.random.default_rng(9)
    lam = rng.standard_normal(Sg.shape)
    lam_t, dtau, dbin, dein = oracle.adjoint_step(p, Sg, lam)
    sv = Solver(s)
    g = upload_g(sv, Sg)
    ln = upload_lam(sv, lam)
    lo = torch.full_like(ln, float("nan"))
    dt = torch.zeros(s.batch, dtype=torch.float64, device=sv.device)
    db = torch.zeros(3, dtype=torch.float64, device=sv.device)
    de = torch.zeros(1, dtype=torch.float64, device=sv.device)
    sv.adjoint_step(g, ln, lo, dt, db, de)
    got = sv.unpack(lo).cpu().numpy()
    assert np.isfinite(got).all(), "some lambda_t entry was never written"
    assert rel(got, lam_t) <= 1e-12
    assert rel(dt.cpu().numpy(), dtau) <= 1e-12
    if any(b == ri.INFLOW for ax in s.bc for b in ax):
        assert rel(db.cpu().numpy(), dbin) <= 1e-12
        assert rel(de.cpu().numpy(), np.array([dein])) <= 1e-12
    # lam_next is left unmodified
    assert np.array_equal(sv.unpack(ln).cpu().numpy(), lam)
    sv.close()


@pytest.mark.parametrize("name", ["inflow_outflow_obstacle", "tachyon"])
def test_moments_and_init_adjoint_match_oracle(name):
    from paper_0912_2913_amd.solver import Solver

    s = setups()[name]
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, 2)
    Sg = np.ascontiguousarray(S[1])
    rng = np.random.default_rng(10)
    dLde = rng.standard_normal(s.cells)
    dLdb = rng.standard_normal((3, s.cells))
    lam_ref = oracle.moments_adjoint(p, Sg, dLde, dLdb)
    sv = Solver(s)
    lam = sv.new_lam()
    sv.moments_adjoint(upload_g(sv, Sg), torch.as_tensor(dLde, device=sv.device),
                       torch.as_tensor(dLdb, device=sv.device), lam)
    assert rel(sv.unpack(lam).cpu().numpy(), lam_ref) <= 1e-12
    lam0 = rng.standard_normal((19, s.cells))
    de0_ref, db0_ref, dbin_ref, dein_ref = oracle.init_adjoint(p, s.e0, s.beta0, lam0)
    de0 = torch.empty(s.cells, dtype=torch.float64, device=sv.device)
    db0 = torch.empty((3, s.cells), dtype=torch.float64, device=sv.device)
    dbin = torch.zeros(3, dtype=torch.float64, device=sv.device)
    dein = torch.zeros(1, dtype=torch.float64, device=sv.device)
    sv.init_adjoint(upload_lam(sv, lam0), de0, db0, dbin, dein)
    assert rel(de0.cpu().numpy(), de0_ref) <= 1e-12
    assert rel(db0.cpu().numpy(), db0_ref) <= 1e-12
    if any(b == ri.INFLOW for ax in s.bc for b in ax):
        assert rel(dbin.cpu().numpy(), dbin_ref) <= 1e-12
        assert rel(dein.cpu().numpy(), np.array([dein_ref])) <= 1e-12
    sv.close()


def _loss_arrays(s, seed=0):
    rng = np.random.default_rng(seed)
    C = s.cells
    return (rng.uniform(0.5, 1.5, C), rng.uniform(0.2, 1.0, C), rng.standard_normal(C) * 0.1,
            rng.standard_normal((3, C)) * 0.1)


def _gpu_gradient(s, steps, checkpoint, seed=0):
    from paper_0912_2913_amd.autograd import rlb_run

    dev = "cuda:0"
    f64 = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), device=dev, requires_grad=True)
    tau = f64(s.tau)
    e_in = f64([s.inflow[1]])
    b_in = f64(s.inflow[2:5])
    e0 = f64(s.e0)
    b0 = f64(s.beta0)
    e, b = rlb_run(s, steps, tau, e_in, b_in, e0, b0, checkpoint=checkpoint)
    a, t, be, bb = [torch.as_tensor(v, device=dev) for v in _loss_arrays(s, seed)]
    m = torch.ones(s.cells, dtype=torch.bool, device=dev) if s.solid is None else \
        torch.as_tensor(s.solid == 0, device=dev)
    L = ((a * (e - t) ** 2 + be * e)[m]).sum() + ((bb * b)[:, m]).sum()
    L.backward()
    return float(L), tau.grad.cpu().numpy(), e_in.grad.cpu().numpy(), b_in.grad.cpu().numpy(), \
        e0.grad.cpu().numpy(), b0.grad.cpu().numpy()


@pytest.mark.parametrize("name,steps", [("tube_batch", 60), ("inflow_outflow_obstacle", 25)])
def test_checkpointed_gradient_matches_oracle_reverse_sweep(name, steps):
    s = setups()[name]
    p = problem(s)
    a, t, be, bb = _loss_arrays(s)
    G = oracle.gradient(p, s.e0, s.beta0, steps, oracle.Loss(a, t, be, bb))
    L, gt, gei, gbi, ge0, gb0 = _gpu_gradient(s, steps, "sqrt")
    assert L == pytest.approx(G.loss, rel=1e-12)
    assert rel(gt, G.tau) <= 1e-10
    assert rel(ge0, G.e0) <= 1e-10
    assert rel(gb0, G.beta0) <= 1e-10
    if any(b == ri.INFLOW for ax in s.bc for b in ax):
        assert rel(gbi, G.beta_in) <= 1e-10
        assert rel(gei, np.array([G.e_in])) <= 1e-10


def test_checkpointed_equals_store_all_bitwise():
    s = setups()["inflow_outflow_obstacle"]
    r1 = _gpu_gradient(s, 30, "sqrt")
    r2 = _gpu_gradient(s, 30, "store_all")
    r3 = _gpu_gradient(s, 30, 7)
    r4 = _gpu_gradient(s, 30, "3level")  # segments of 16 split into sub-segments of 4
    for x, y, z, w in zip(r1[1:], r2[1:], r3[1:], r4[1:]):
        assert np.array_equal(x, y) and np.array_equal(x, z) and np.array_equal(x, w)


def test_overlapped_recompute_equals_sequential_bitwise():
    """The sqrt(T) reverse pass with each segment's recompute on a second solver
    and stream (overlapped with the previous segment's sweep) gives the same
    gradient bit for bit as the pass that recomputes and sweeps in turn."""
    import paper_0912_2913_amd.autograd as A

    s = setups()["inflow_outflow_obstacle"]
    saved = A.OVERLAP_RECOMPUTE
    try:
        A.OVERLAP_RECOMPUTE = True
        r1 = _gpu_gradient(s, 40, 5)
        A.OVERLAP_RECOMPUTE = False
        r2 = _gpu_gradient(s, 40, 5)
    finally:
        A.OVERLAP_RECOMPUTE = saved
    assert r1[0] == r2[0]
    for x, y in zip(r1[1:], r2[1:]):
        assert np.array_equal(x, y)


def test_gradient_matches_central_differences_fp64():
    """tau and e0-direction derivatives vs central FD of GPU FP64 forward runs."""
    from paper_0912_2913_amd.autograd import rlb_run

    s = setups()["tube_batch"]
    steps = 80
    a, t, _, _ = _loss_arrays(s, 3)
    dev = "cuda:0"
    at, tt = torch.as_tensor(a, device=dev), torch.as_tensor(t, device=dev)

    def loss(tau, e0):
        with torch.no_grad():
            e, _ = rlb_run(s, steps, tau=torch.as_tensor(tau, device=dev),
                           e0=torch.as_tensor(e0, device=dev))
            return float((at * (e - tt) ** 2).sum())

    tau = torch.tensor(s.tau, device=dev, requires_grad=True)
    e0 = torch.tensor(s.e0, device=dev, requires_grad=True)
    e, _ = rlb_run(s, steps, tau=tau, e0=e0)
    (at * (e - tt) ** 2).sum().backward()
    h = 1e-6
    for b in range(s.batch):
        d = np.zeros(s.batch)
        d[b] = h
        fd = (loss(s.tau + d, s.e0) - loss(s.tau - d, s.e0)) / (2 * h)
        assert float(tau.grad[b]) == pytest.approx(fd, rel=1e-6)
    v = np.random.default_rng(4).standard_normal(s.cells) * 1e-2
    fd = (loss(s.tau, s.e0 + h * v) - loss(s.tau, s.e0 - h * v)) / (2 * h)
    assert float((e0.grad.cpu().numpy() * v).sum()) == pytest.approx(fd, rel=1e-6)


# ---------------------------------------------------------------------------
# Loop entry points: one call per segment instead of one per step.

def bits(t: torch.Tensor) -> torch.Tensor:
    """Bit pattern of a tensor (bitwise comparison that also holds for NaN
    payloads in never-written padding)."""
    return t.contiguous().view(torch.uint8)


def _state_after(s, steps):
    p = problem(s)
    S = oracle.init(p, s.n0, s.e0, s.beta0)
    oracle.run(p, S, steps)
    return np.ascontiguousarray(S[1])


@pytest.mark.parametrize("storage", [ri.F64, ri.F32DEV, ri.BF16DEV])
def test_advance_and_trajectory_equal_step_g_chain_bitwise(storage):
    from dataclasses import replace

    from paper_0912_2913_amd.solver import Solver

    s = replace(setups()["inflow_outflow_obstacle"], storage=storage, e_ref=1.0)
    sv = Solver(s)
    fl = torch.as_tensor(s.solid == 0, device=sv.device)  # solid entries are never written
    g0 = sv.g_state().clone()
    chain = [g0.clone()]
    for _ in range(6):
        nxt = sv.new_g()
        sv.step_g(chain[-1], nxt)
        chain.append(nxt)
    tmp = sv.new_g()
    for n in (0, 1, 2, 5, 6):
        dst = sv.new_g().fill_(7)
        sv.advance_g(g0, dst, tmp, n)
        assert torch.equal(bits(sv.unpack(dst)[:, fl]), bits(sv.unpack(chain[n])[:, fl])), n
    assert torch.equal(bits(g0), bits(chain[0]))  # the source is read only
    seq = sv.new_g_seq(7)
    seq[0].copy_(g0)
    seq[1:].fill_(3)
    sv.trajectory_g(seq, 5)
    for j in range(5):
        assert torch.equal(bits(sv.unpack(seq[j])[:, fl]), bits(sv.unpack(chain[j])[:, fl])), j
    assert bool((seq[5:] == 3).all())  # blocks beyond n untouched
    sv.close()


@pytest.mark.parametrize("name", ["inflow_outflow_obstacle", "tube_batch"])
def test_adjoint_sweep_equals_pending_adjoint_steps(name):
    """A sweep of n steps = n rlb_adjoint_step calls whose partials stay pending
    until the last call passes gradient pointers: lambda and gradients bitwise.
    Against steps flushed one by one: lambda bitwise, gradients to rounding."""
    from paper_0912_2913_amd.solver import Solver

    s = setups()[name]
    sv = Solver(s)
    n = 5
    seq = sv.new_g_seq(n)
    seq[0].copy_(upload_g(sv, _state_after(s, 2)))
    sv.trajectory_g(seq, n)
    rng = np.random.default_rng(11)
    lam_T = upload_lam(sv, rng.standard_normal((19, s.cells)))
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=sv.device)

    la, lb = lam_T.clone(), torch.full_like(lam_T, float("nan"))
    res = sv.adjoint_sweep(seq, n, la, lb)
    assert res is (lb if n % 2 == 0 else la)  # n reader-form steps, then the gather
    g_sw = (z(s.batch), z(3), z(1))
    sv.adjoint_flush(*g_sw)

    a, b = lam_T.clone(), torch.full_like(lam_T, float("nan"))
    g_pe = (z(s.batch), z(3), z(1))
    for j in range(n - 1, -1, -1):
        sv.adjoint_step(seq[j], a, b, *(g_pe if j == 0 else (None, None, None)))
        a, b = b, a
    assert torch.equal(sv.unpack(a), sv.unpack(res))
    for x, y in zip(g_sw, g_pe):
        assert torch.equal(x, y)

    a, b = lam_T.clone(), torch.full_like(lam_T, float("nan"))
    g_ea = (z(s.batch), z(3), z(1))
    for j in range(n - 1, -1, -1):
        sv.adjoint_step(seq[j], a, b, *g_ea)
        a, b = b, a
    for x, y in zip(g_sw, g_ea):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1e-300)
    sv.close()


@pytest.mark.parametrize("name", ["inflow_outflow_obstacle", "outflow_corners",
                                  "inflow_x_solid_on_outflow_face", "thin_outflow_axis_and_inflow",
                                  "tube_batch"])
def test_reader_form_segments_equal_step_by_step(name):
    """Segments chained in reader form (a checkpoint read in place plus its
    successors per call, one gather at the end) give the lambda and the
    parameter partials of single natural rlb_adjoint_step calls bit for bit."""
    from paper_0912_2913_amd._lib import RLBError
    from paper_0912_2913_amd.solver import Solver

    s = setups()[name]
    sv = Solver(s)
    T = 9
    st = sv.new_g_seq(T)
    st[0].copy_(upload_g(sv, _state_after(s, 2)))
    sv.trajectory_g(st, T)
    rng = np.random.default_rng(14)
    lam_T = upload_lam(sv, rng.standard_normal((19, s.cells)))
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=sv.device)
    a, b = lam_T.clone(), sv.new_lam()
    g_ref = (z(s.batch), z(3), z(1))
    for j in range(T - 1, -1, -1):
        sv.adjoint_step(st[j], a, b, *(g_ref if j == 0 else (None, None, None)))
        a, b = b, a
    lam_ref = sv.unpack(a)
    # segments [6, 9), [2, 6), [1, 2), [0, 1): natural in, reader form between
    la, lb = lam_T.clone(), sv.new_lam()
    reader = False
    for lo, hi in ((6, 9), (2, 6), (1, 2), (0, 1)):
        seq = st[lo + 1:hi].contiguous() if hi - lo > 1 else None
        res = sv.adjoint_segment(st[lo], seq, hi - lo, la, lb, in_reader=reader, out_reader=True)
        la, lb = res, (lb if res is la else la)
        reader = True
    sv.lam_gather(la, lb)
    g_seg = (z(s.batch), z(3), z(1))
    sv.adjoint_flush(*g_seg)
    assert torch.equal(sv.unpack(lb), lam_ref)
    for x, y in zip(g_seg, g_ref):
        assert torch.equal(x, y)
    # n = 0: a reader-form lambda is gathered; a natural one is returned as is
    res = sv.adjoint_segment(None, None, 0, la, lb, in_reader=True)
    assert res is lb
    assert sv.adjoint_segment(None, None, 0, la, lb) is la
    with pytest.raises(RLBError):
        sv.adjoint_segment(None, None, 0, la, lb, out_reader=True)
    sv.close()


def test_flush_discards_and_empty_flush_is_a_no_op():
    from paper_0912_2913_amd.solver import Solver

    s = setups()["inflow_outflow_obstacle"]
    g = None
    rng = np.random.default_rng(12)
    lam = rng.standard_normal((19, s.cells))
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda:0")

    def one_step(sv, pending_first):
        nonlocal g
        g = upload_g(sv, _state_after(s, 1)) if g is None else g
        ln, lo = upload_lam(sv, lam), sv.new_lam()
        if pending_first:
            sv.adjoint_step(g, ln, lo)  # pending ...
            sv.adjoint_flush()          # ... and discarded
        out = (z(s.batch), z(3), z(1))
        sv.adjoint_flush(*out)          # nothing pending: no change
        assert all(float(t.abs().max()) == 0.0 for t in out)
        sv.adjoint_step(g, ln, lo, *out)
        return [t.cpu().numpy() for t in out]

    sv1 = Solver(s)
    r1 = one_step(sv1, True)
    sv1.close()
    sv2 = Solver(s)
    r2 = one_step(sv2, False)
    sv2.close()
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)


def test_loop_entry_points_reject_bad_arguments():
    from paper_0912_2913_amd._lib import RLBError
    from paper_0912_2913_amd.solver import Solver

    s = setups()["outflow_corners"]
    sv = Solver(s)
    a, b, c = sv.new_g(), sv.new_g(), sv.new_g()
    for args in ((a, b, c, -1), (a, a, c, 2), (a, b, a, 2), (a, b, b, 2)):
        with pytest.raises(RLBError):
            sv.advance_g(*args)
    seq = sv.new_g_seq(3)
    with pytest.raises(ValueError):
        sv.trajectory_g(seq, 0)
    with pytest.raises(ValueError):
        sv.trajectory_g(seq, 4)
    la = sv.new_lam()
    with pytest.raises(RLBError):
        sv.adjoint_sweep(seq, 2, la, la)
    sv.close()


def test_graph_replays_match_step_by_step_launches():
    """Loop entry points of 4 or more steps launch directly the first time a
    call's arguments are seen, capture a graph the second time and replay it
    afterwards: every repetition, with other work and synchronisations in
    between, matches the step-by-step result bitwise (advance, trajectory,
    sweep; the sweep's partials too)."""
    from paper_0912_2913_amd.solver import Solver

    s = setups()["inflow_outflow_obstacle"]
    sv = Solver(s)
    g0 = upload_g(sv, _state_after(s, 2))
    ref = [g0.clone()]
    for _ in range(6):
        nxt = sv.new_g().zero_()
        sv.step_g(ref[-1], nxt)
        ref.append(nxt)
    fl = torch.as_tensor(s.solid == 0, device=sv.device)
    dst, tmp = sv.new_g(), sv.new_g()
    seq = sv.new_g_seq(6)
    rng = np.random.default_rng(13)
    lam_T = upload_lam(sv, rng.standard_normal((19, s.cells)))
    z = lambda k: torch.zeros(k, dtype=torch.float64, device=sv.device)
    # the step-by-step sweep (single rlb_adjoint_step calls) as the reference
    seq[0].copy_(g0)
    sv.trajectory_g(seq, 3)  # < 4 steps: launched step by step
    seq_ref = seq.clone()
    for j in range(3, 6):
        sv.step_g(seq_ref[j - 1], seq_ref[j])
    a, b = lam_T.clone(), sv.new_lam()
    g_ref = (z(s.batch), z(3), z(1))
    for j in range(5, -1, -1):
        sv.adjoint_step(seq_ref[j], a, b, *(g_ref if j == 0 else (None, None, None)))
        a, b = b, a
    lam_ref = sv.unpack(a).cpu()
    la, lb = sv.new_lam(), sv.new_lam()
    for rep in range(4):
        dst.fill_(float(rep))
        sv.advance_g(g0, dst, tmp, 6)
        assert torch.equal(bits(sv.unpack(dst)[:, fl]), bits(sv.unpack(ref[6])[:, fl])), rep
        seq.fill_(-1.0)
        seq[0].copy_(g0)
        sv.trajectory_g(seq, 6)
        for j in range(6):
            assert torch.equal(bits(sv.unpack(seq[j])[:, fl]), bits(sv.unpack(seq_ref[j])[:, fl])), (rep, j)
        torch.cuda.synchronize()
        _ = (dst * 2).sum().item()  # unrelated eager work between replays
        la.copy_(lam_T)
        lb.fill_(float("nan"))
        res = sv.adjoint_sweep(seq, 6, la, lb)
        g_sw = (z(s.batch), z(3), z(1))
        sv.adjoint_flush(*g_sw)
        assert torch.equal(sv.unpack(res).cpu(), lam_ref), rep
        for x, y in zip(g_sw, g_ref):
            assert torch.equal(x, y), rep
    sv.close()


def decoded_g(sv, s) -> np.ndarray:
    """The solver's current g block decoded to FP64 [19][cells]: the stored
    values, plus the rest equilibrium R at (n_ref, e_ref) for the deviation
    storages (R from the oracle's equilibria at beta = 0); zeros on solid cells."""
    g = sv.unpack(sv.g_state()).double().cpu().numpy()
    if s.storage in (ri.F32DEV, ri.F16DEV, ri.BF16DEV):
        _, R = oracle.equilibria(s.n_ref, s.e_ref, np.zeros(3), s.c_l, s.kappa)
        g = g + R[:, None]
    if s.solid is not None:
        g[:, s.solid.reshape(-1) != 0] = 0.0
    return np.ascontiguousarray(g)


STORAGES = [ri.F32, ri.F32DEV, ri.F16DEV, ri.BF16DEV]


@pytest.mark.parametrize("storage", STORAGES, ids=[ri.STORAGE_NAMES[v] for v in STORAGES])
@pytest.mark.parametrize("name", ["inflow_outflow_obstacle", "outflow_corners",
                                  "inflow_x_solid_on_outflow_face", "tachyon"])
def test_reverse_entry_points_every_storage_match_oracle(name, storage):
    """The reverse arithmetic is FP64 for every storage: on the GPU's own state
    (a few forward steps in the storage format), decoded to FP64, the adjoint
    step, the moment adjoint and the initial-state adjoint match the oracle's
    complex-step transposes at 1e-12."""
    from paper_0912_2913_amd.solver import Solver

    s = setups()[name].with_(storage=storage, n_ref=0.9, e_ref=1.05)
    p = problem(s)
    sv = Solver(s)
    sv.step(3)
    Sg = decoded_g(sv, s)
    rng = np.random.default_rng(21)
    lam = rng.standard_normal(Sg.shape)
    lam_t, dtau, dbin, dein = oracle.adjoint_step(p, Sg, lam)
    g = sv.g_state().clone()
    ln = upload_lam(sv, lam)
    lo = torch.full_like(ln, float("nan"))
    dt = torch.zeros(s.batch, dtype=torch.float64, device=sv.device)
    db = torch.zeros(3, dtype=torch.float64, device=sv.device)
    de = torch.zeros(1, dtype=torch.float64, device=sv.device)
    sv.adjoint_step(g, ln, lo, dt, db, de)
    got = sv.unpack(lo).cpu().numpy()
    assert rel(got, lam_t) <= 1e-12
    assert rel(dt.cpu().numpy(), dtau) <= 1e-12
    if any(b == ri.INFLOW for ax in s.bc for b in ax):
        assert rel(db.cpu().numpy(), dbin) <= 1e-12
        assert rel(de.cpu().numpy(), np.array([dein])) <= 1e-12
    dLde = rng.standard_normal(s.cells)
    dLdb = rng.standard_normal((3, s.cells))
    lam_ref = oracle.moments_adjoint(p, Sg, dLde, dLdb)
    lamT = sv.new_lam()
    sv.moments_adjoint(g, torch.as_tensor(dLde, device=sv.device),
                       torch.as_tensor(dLdb, device=sv.device), lamT)
    assert rel(sv.unpack(lamT).cpu().numpy(), lam_ref) <= 1e-12
    de0_ref, db0_ref, dbin_ref, dein_ref = oracle.init_adjoint(p, s.e0, s.beta0, lam)
    de0 = torch.empty(s.cells, dtype=torch.float64, device=sv.device)
    db0 = torch.empty((3, s.cells), dtype=torch.float64, device=sv.device)
    dbi = torch.zeros(3, dtype=torch.float64, device=sv.device)
    dei = torch.zeros(1, dtype=torch.float64, device=sv.device)
    sv.init_adjoint(ln, de0, db0, dbi, dei)
    assert rel(de0.cpu().numpy(), de0_ref) <= 1e-12
    assert rel(db0.cpu().numpy(), db0_ref) <= 1e-12
    sv.close()
