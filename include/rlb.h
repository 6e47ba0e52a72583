/*
 * rlb.h -- C ABI of the MI355X relativistic lattice Boltzmann (RLB) library.
 *
 * The library advances the two-population D3Q19 scheme of Mendoza, Boghosian,
 * Herrmann and Succi, "Lattice Boltzmann scheme for relativistic fluids"
 * (arXiv:0912.2913): a number population f_i and an energy-momentum
 * population g_i per cell and velocity, relaxed by one BGK time tau
 * (eqs. lbe1, lbe2) toward the ultra-relativistic equilibria
 * (eqs. equil1s, equil2as, equil2bs; for P = kappa e with kappa != 1/3 the
 * general ones, eqs. equil1, equil2a, equil2b), with (n, e, beta) recovered
 * from the macroscopic constraints n gamma = sum f_i, (e+P) gamma^2 - P =
 * sum g_i, (e+P) gamma^2 beta = sum g_i c_i closed by the equation of state.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: c = 1; c_i = c_l e_i with e_i the integer D3Q19 vectors; one cell
 *    = dx, one step = dt = dx / c_l; tau is in units of dt (omega = 1/tau).
 *  - Cell index: cell = ((b*nz + z)*ny + y)*nx + x, x fastest; b = instance.
 *    cells = batch*nz*ny*nx.
 *  - Population buffer ("state"): two population blocks, f then g, of
 *    19*q_stride elements each, q_stride = cells rounded up to a multiple of
 *    64 (see rlb_buffer_layout).  Inside a block the cells are grouped in
 *    bricks of 64 consecutive cells, each brick holding its 19 directions
 *    one after another: element (q, cell) of a block is at
 *      (cell / 64) * 19 * 64 + q * 64 + cell % 64,
 *    and the g block starts at element 19*q_stride.  A "g block" is that
 *    second half on its own (any g state, e.g. a checkpoint).
 *    Element type by storage: RLB_F64 double; RLB_F32 float; RLB_F32DEV float,
 *    RLB_F16DEV IEEE binary16, RLB_BF16DEV bfloat16, the *DEV forms holding
 *    the deviation S_i - R_i from the rest equilibrium R at (n_ref, e_ref).
 *  - Velocity ordering: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..10 = (1,1,0),
 *    (-1,-1,0),(1,-1,0),(-1,1,0); 11..14 = (1,0,1),(-1,0,-1),(1,0,-1),
 *    (-1,0,1); 15..18 = (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 *  - Stored state = post-collision populations S_t; one step computes
 *    S_{t+1}(x) = collide(pull(S_t))(x).  Fields at time t are the moments of
 *    S_t (the collision conserves sum f, sum g and sum g c_i).
 *  - Boundaries (per face): PERIODIC wraps; OUTFLOW copies (pull source
 *    clamped into the domain); INFLOW holds the face plane at the equilibrium
 *    of (inflow_n, inflow_e, inflow_beta).  Solid cells reflect by half-way
 *    bounce-back and are never updated.
 *  - In-place streaming (rlb_params.inplace = 1): the solver keeps one state
 *    buffer (pop_a; pop_b may be NULL) and alternates two kernels.  After an
 *    even number of steps pop_a holds S_t with S_t(x)_q at slot opp(q) of x
 *    (the "swapped" layout: element (pop, opp(q), x) in the formula above);
 *    after an odd number it holds the pulled, pre-collision values of the
 *    next step, P(x)_q at slot q, from which S_t is not recoverable
 *    everywhere.  rlb_moments and rlb_transport then need an even step count;
 *    the g-only, reverse-mode and held-eta/s entry points are not available.
 *    Same HBM traffic per step, half the state memory.
 *  - Adjoint buffers ("lambda"): one block in the same brick layout, double
 *    for every storage.  Natural form: lambda(x)_q = dL / dS(x)_q.  Reader
 *    form (see rlb_adjoint_segment): R(r)_q = the contribution of cell r's
 *    update through its pull of direction q, stored at r; the natural form
 *    is its gather, lambda(x)_p = R(x + e_p)_p (or R(x)_opp(p) when x's pull
 *    of opp(p) bounces off a solid) plus R(r)_p of every cell r whose pull
 *    of p is clamped onto x by an outflow face.
 *  - Device pointers address memory on the solver's device; every call that
 *    launches work is asynchronous on the stream given to rlb_init unless its
 *    comment says it synchronises.  Nothing throws across the ABI.
 *  - Errors: RLB_EINVAL = invalid argument, nothing launched;
 *    RLB_EDEVICE = a HIP call failed; rlb_last_error() gives details.
 */
#ifndef RLB_H
#define RLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlb_solver rlb_solver; /* opaque, owned by the library */

typedef enum {
  RLB_OK = 0,
  RLB_EINVAL = -1,
  RLB_ENOMEM = -2,
  RLB_EDEVICE = -3,
  RLB_EUNPHYSICAL = -4
} rlb_status;

typedef enum { RLB_BC_PERIODIC = 0, RLB_BC_OUTFLOW = 1, RLB_BC_INFLOW = 2 } rlb_bc;

typedef enum {
  RLB_F64 = 0,
  RLB_F32 = 1,
  RLB_F32DEV = 2,
  RLB_F16DEV = 3,
  RLB_BF16DEV = 4
} rlb_storage;

/* Type of the collision arithmetic (moment sums, equilibria, relaxation); the
 * moment inversion is FP64 always.  AUTO = FP64 for RLB_F64/F32/F32DEV and
 * FP32 for the 16-bit storages.  F32_MOM64 (4-byte storages only): FP32
 * equilibria and relaxation with FP64 moments: the pre-collision sums
 * accumulated in FP64, and the FP32 g equilibrium corrected by
 * w_i (dE + 3 e_i . dm) so that its FP64-summed moments equal them (FP32
 * coefficients would otherwise bias the conserved sums the same way every
 * step).  FP32 collision is not offered with RLB_F64 storage, nor FP64
 * collision with 16-bit storage. */
typedef enum {
  RLB_COLLIDE_AUTO = 0,
  RLB_COLLIDE_F32 = 1,
  RLB_COLLIDE_F64 = 2,
  RLB_COLLIDE_F32_MOM64 = 3
} rlb_collide;

/* Problem statement (shock-tube and obstacle sections of the paper: domain,
 * lattice speed c_l, fixed obstacle, inflow state; equation of state). */
typedef struct {
  int32_t nx, ny, nz, batch; /* extents (>= 1); batch independent lattices       */
  double c_l;                /* lattice speed in units of c (> 0)                */
  int32_t bc[3][2];          /* [axis x,y,z][low, high face] : rlb_bc            */
  double inflow_n, inflow_e; /* inflow state (used when a face is INFLOW)        */
  double inflow_beta[3];
  int32_t storage;           /* rlb_storage                                      */
  double n_ref, e_ref;       /* rest reference of the *DEV storages              */
  int32_t collide;           /* rlb_collide                                      */
  double kappa;              /* equation of state P = kappa e, 0 < kappa <= 1;   */
                             /* 0 selects 1/3 (e = 3P, the paper's simulations)  */
  int32_t inplace;           /* 1: one state buffer, in-place streaming (below)  */
} rlb_params;

/* Layout of one population buffer for these parameters: q_stride (cells
 * rounded up to 64, i.e. 64 * number of bricks) and the byte size of a full
 * f+g buffer (2*19*q_stride*elem).
 * Either output may be NULL.  Host-only, no device work. */
rlb_status rlb_buffer_layout(const rlb_params *p, int64_t *q_stride, int64_t *state_bytes);

/* Create a solver and write the initial state S_0 into pop_a.
 *  tau   : host [batch], each > 1/2 (eta = (4/9) gamma^2 e (tau - dt/2) c_l^2 > 0).
 *  solid : device uint8 [cells] (nonzero = solid) or NULL; copied.
 *  n0, e0: device double [cells]; beta0: device double [3][cells].  Read
 *          during this call only.  S_0 = (f^eq(n0 gamma0, beta0),
 *          g^eq(e0, beta0)) on fluid cells, the inflow equilibrium on inflow
 *          cells, zeros on solid cells (in both pop_a and pop_b).
 *  pop_a, pop_b: caller-owned device buffers of state_bytes each, aliased by
 *          the solver until rlb_destroy; the steps ping-pong between them
 *          (in-place streaming: pop_a only, pop_b unused and may be NULL).
 *  stream: hipStream_t (NULL = default stream) for all of the solver's work.
 * Validation: extents >= 1 (>= 2 on non-periodic axes); periodic on both or
 * neither face of an axis; at most one INFLOW face; inflow_e > 0 and
 * |inflow_beta| < 1 when a face is INFLOW; c_l > 0; e_ref > 0 for *DEV;
 * cells <= 2^31 - 64.  Library-owned device memory: a copy of tau, a cell
 * class mask, small reduction and counter buffers. */
rlb_status rlb_init(rlb_solver **out, const rlb_params *p, const double *tau,
                    const uint8_t *solid, const double *n0, const double *e0,
                    const double *beta0, void *pop_a, void *pop_b, void *stream);

/* Advance nsteps (>= 0) full f+g steps (eqs. lbe1 and lbe2 with pull
 * streaming and the boundary rules above).  Asynchronous. */
rlb_status rlb_step(rlb_solver *h, int32_t nsteps);

/* One step of the g population alone from g_src to g_dst (g blocks,
 * 19*q_stride elements, distinct).  f never enters (e, beta), so this is the exact
 * g part of rlb_step; used to recompute states in a reverse sweep.  Solid
 * cells' entries are written with the value rlb_init gives them (encoded
 * zero), inflow-plane cells with the inflow equilibrium; the padding beyond
 * the cells is not written (no step reads it). */
rlb_status rlb_step_g(rlb_solver *h, const void *g_src, void *g_dst);

/* n (>= 0) steps of the g population alone, as n calls of rlb_step_g, from
 * g_src to g_dst, ping-ponging through g_tmp so that the last step lands in
 * g_dst (n = 0 copies g_src to g_dst).  g_src is read only; g_tmp (needed
 * for n > 1) is overwritten; the three buffers are distinct g blocks.  Solid
 * and padding entries as in rlb_step_g (copied when n = 0).  One
 * call replaces n host round trips (the checkpointed forward sweep).
 * Loop calls (this one, rlb_trajectory_g, rlb_adjoint_sweep) of n >= 4 are
 * replayed from a HIP graph that the library captures on the second call
 * with the same buffers and n; the graph holds the pointers, not the data.
 * rlb_set_tau_field and rlb_hold_eta_over_s drop the captured graphs. */
rlb_status rlb_advance_g(rlb_solver *h, const void *g_src, void *g_dst, void *g_tmp,
                         int32_t n);

/* Recompute a stretch of g states in place: g_seq holds n (>= 1) g blocks,
 * block j at byte offset j * seq_stride (seq_stride >= the g block's bytes);
 * block 0 is read, blocks 1 .. n-1 are overwritten with
 * block j = rlb_step_g(block j-1).  Used to restore a segment of a
 * checkpointed trajectory before its reverse sweep. */
rlb_status rlb_trajectory_g(rlb_solver *h, void *g_seq, int64_t seq_stride, int32_t n);

/* Device pointer of the buffer that holds the current state S_t. */
rlb_status rlb_current(rlb_solver *h, void **state);

/* Fields of the current state: n, e [cells], beta [3][cells] (device double,
 * any may be NULL; zeros on solid cells).  sums: host double [batch][5] =
 * (sum f, sum g, sum g c_x, sum g c_y, sum g c_z) over non-solid cells,
 * reduced in a fixed order in FP64 (bitwise reproducible), or NULL.  With
 * sums != NULL the call synchronises the stream.  In-place streaming:
 * RLB_EINVAL after an odd number of steps (S_t is not stored then). */
rlb_status rlb_moments(rlb_solver *h, double *n, double *e, double *beta, double *sums);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * fields of rlb_moments, and the same conservation sums, bit for bit, but
 * written to sums = device double [batch][5] (or NULL) on the solver's
 * stream, without synchronising and without allocating anything.  The
 * per-workgroup partials of the sums live in a static device workspace of
 * 8 MiB that the library holds on every device it runs on until the process
 * ends (its address is looked up once per device by rlb_init): at most
 * 8 MiB / 40 B = 209715 workgroups of 256 cells, each instance's cells
 * rounded up to whole workgroups (about 53.6 million cells in one
 * instance).  Larger lattices with sums != NULL return RLB_EINVAL with
 * nothing launched.  Every call on one device shares that workspace:
 * calls whose work overlaps on one device (several streams, several
 * threads) race; calls ordered on one stream do not.  Each call rewrites
 * every partial it reads, so nothing needs clearing between calls.
 * n, e, beta: as rlb_moments (device double, any may be NULL).  In-place
 * streaming: RLB_EINVAL after an odd number of steps. */
rlb_status rlb_moments_noalloc(rlb_solver *h, double *n, double *e, double *beta, double *sums);

/* Fields e [cells] and beta [3][cells] (device double, either may be NULL)
 * of a g block (any state of the g population, e.g. one from rlb_step_g):
 * the constraints for (e, beta) involve g alone.  Zeros on solid cells. */
rlb_status rlb_fields_g(rlb_solver *h, const void *g_state, double *e, double *beta);

/* Counters of the steps run since the last call (synchronises): counts[0] =
 * unphysical g updates (no real root of the inversion, 4E^2 - 3|M|^2 <= 0
 * for e = 3P; e <= 0, |beta| >= 1 or NaN);
 * counts[1] = f updates whose equilibrium had a non-positive component
 * (some c_i.beta <= -c_l^2/3, the paper's positivity bound).  Resets both.
 * Returns RLB_EUNPHYSICAL when counts[0] > 0. */
rlb_status rlb_counters(rlb_solver *h, int64_t counts[2]);

/* Flags of rlb_adjoint_segment. */
#define RLB_LAM_IN_READER 1  /* lam_a holds lambda in reader form             */
#define RLB_LAM_OUT_READER 2 /* leave the result in reader form (no gather)   */

/* One reverse step of the g population (the transpose of the linearised
 * update of eq. lbe2 with its streaming and boundary rules):
 *   lam_out = (d S_{t+1} / d S_t)^T lam_next,
 * where S_{t+1} = step(S_t) with S_t = g_state_t (a g block), for the
 * solver's equation of state (any kappa).  lam_next and
 * lam_out are device double blocks (brick layout) for every storage, distinct;
 * lam_out is overwritten, lam_next is not modified.  The step's parameter
 * contributions,
 *   dL_dtau[batch]  += lam_next . d S_{t+1} / d tau,
 *   dL_dbeta_in[3], dL_de_in[1] += lam_next . d S_{t+1} / d(inflow state),
 * are first added to per-workgroup partials held by the solver, in step
 * order.  When any of the three (device double) gradient pointers is
 * non-NULL the pending partials of this and all earlier unreduced steps are
 * reduced into them (as rlb_adjoint_flush); with all three NULL they stay
 * pending.  Reductions run in a fixed order, so results are bitwise
 * reproducible and independent of how a sweep is split into calls.  The
 * step's reader form passes through a library-owned lambda block (allocated
 * on the first call), then is gathered into lam_out. */
rlb_status rlb_adjoint_step(rlb_solver *h, const void *g_state_t, const void *lam_next,
                            void *lam_out, double *dL_dtau, double *dL_dbeta_in,
                            double *dL_de_in);

/* n (>= 0) reverse steps in one call: for j = n-1 down to 0, one
 * rlb_adjoint_step with g_state_t = block j of g_seq (layout as in
 * rlb_trajectory_g) and all gradient pointers NULL (the contributions stay
 * pending).  lam_a holds the (natural) adjoint after the last state on entry;
 * lam_a and lam_b (distinct device double lambda blocks) are both
 * overwritten, and *lam_result (host) receives whichever of the two holds
 * lambda after block 0: lam_b when n is even and n > 0, else lam_a.  Same as
 * rlb_adjoint_segment with g_first = NULL and flags = 0. */
rlb_status rlb_adjoint_sweep(rlb_solver *h, const void *g_seq, int64_t seq_stride, int32_t n,
                             void *lam_a, void *lam_b, void **lam_result);

/* n (>= 0) reverse steps over a stretch of g states in one call, with lambda
 * passed between calls in either form.  State j of the stretch (j = 0 ..
 * n-1, stepped from n-1 down to 0): with g_first != NULL, state 0 is g_first
 * and state j >= 1 is block j-1 of g_seq (a checkpoint read in place followed
 * by its recomputed successors); with g_first = NULL, state j is block j of
 * g_seq.  lam_a holds lambda after the last state on entry, in reader form
 * when flags has RLB_LAM_IN_READER, else natural.  Each step reads lambda
 * (gathering the reader form with shifted reads) and stores its own
 * contributions aligned, in reader form, into the other of lam_a / lam_b;
 * with RLB_LAM_OUT_READER the result stays in reader form, else it is
 * gathered into the natural form.  *lam_result receives the buffer holding
 * it; both buffers are overwritten.  The parameter contributions stay pending
 * (rlb_adjoint_flush), exactly as n rlb_adjoint_step calls would leave them,
 * and a chain of segments in reader form gives the same lambda bit for bit
 * as step-by-step natural calls.  RLB_EINVAL for n = 0 with
 * RLB_LAM_OUT_READER and a natural input (a natural lambda has no reader
 * form).  Calls of n >= 4 replay captured graphs as rlb_advance_g does. */
rlb_status rlb_adjoint_segment(rlb_solver *h, const void *g_first, const void *g_seq,
                               int64_t seq_stride, int32_t n, void *lam_a, void *lam_b,
                               int32_t flags, void **lam_result);

/* Natural lambda (lam_out, overwritten) from its reader form (lam_reader,
 * unchanged): the gather described at the top of this file; zeros on solid
 * cells.  Distinct device double lambda blocks. */
rlb_status rlb_lam_gather(rlb_solver *h, const void *lam_reader, void *lam_out);

/* Reduce the pending reverse-step partials (fixed order) and add them to
 * dL_dtau[batch], dL_dbeta_in[3], dL_de_in[1] (device double, each may be
 * NULL: that share is discarded).  Afterwards nothing is pending; a call
 * with nothing pending does nothing. */
rlb_status rlb_adjoint_flush(rlb_solver *h, double *dL_dtau, double *dL_dbeta_in,
                             double *dL_de_in);

/* Seed of a reverse sweep: lam_T = (d(e, beta) / d S_T)^T (dL_de, dL_dbeta)
 * per cell, with (e, beta) the fields of the g block g_state_T.  dL_de
 * [cells], dL_dbeta [3][cells]: device double.  lam_T is overwritten. */
rlb_status rlb_moments_adjoint(rlb_solver *h, const void *g_state_T, const double *dL_de,
                               const double *dL_dbeta, void *lam_T);

/* End of a reverse sweep: S_0 = g^eq(e0, beta0) (and the inflow state on
 * inflow cells), so dL_de0 [cells] and dL_dbeta0 [3][cells] are overwritten
 * with (d S_0 / d(e0, beta0))^T lam_0, and dL_dbeta_in, dL_de_in accumulate
 * the inflow cells' share.  e0, beta0: the initial fields given to rlb_init
 * (device double). */
rlb_status rlb_init_adjoint(rlb_solver *h, const double *e0, const double *beta0,
                            const void *lam_0, double *dL_de0, double *dL_dbeta0,
                            double *dL_dbeta_in, double *dL_de_in);

/* Per-cell relaxation times tau(x) (device double [cells], copied), in
 * units of dt, replacing the per-instance tau of rlb_init in every later
 * forward and reverse step; NULL restores the per-instance tau.  The
 * viscosity relation at the end of the equilibrium section,
 * eta = (4/9) gamma^2 e (tau - dt/2) c_l^2, then holds cell by cell.
 * Synchronises (the field is validated): RLB_EINVAL if a non-solid cell's
 * tau is not > 1/2 or NaN, and the previous field (or none) stays in force.
 * While a field is set the reverse steps also accumulate dL/dtau(x) per cell
 * (see rlb_adjoint_flush_tau_field); setting a field clears that
 * accumulator.  Library-owned memory: 16 bytes per cell. */
rlb_status rlb_set_tau_field(rlb_solver *h, const double *tau_cell);

/* Hold eta/s fixed (the shock-tube section characterises its runs by eta/s):
 * with eta_over_s > 0 every later f+g step sets each update's tau from its
 * pre-collision moments of both populations,
 *   tau = 1/2 + 9 (eta/s) s / (4 gamma^2 e c_l),
 *   s = 4n - n ln(n / n_eq), n_eq = d_G T^3 / pi^2, T = e / (3n),
 * overriding the per-instance tau and any tau field.  An update whose rule
 * gives tau <= 1/2 (or NaN) counts as unphysical (rlb_counters).  tau then
 * depends on n, i.e. on f, so rlb_step_g, rlb_advance_g, rlb_trajectory_g,
 * rlb_adjoint_step and rlb_adjoint_sweep return RLB_EINVAL while it is on.
 * eta_over_s = 0 turns it off.  RLB_EINVAL for eta_over_s < 0, d_G <= 0 or
 * non-finite values, and for eta_over_s > 0 with kappa != 1/3 (the rule and
 * T = e/(3n) are those of e = 3P matter).  Host-only (no device work). */
rlb_status rlb_hold_eta_over_s(rlb_solver *h, double eta_over_s, double d_G);

/* Transport quantities of the current state per cell (device double
 * [cells], any may be NULL; zeros on solid cells), from the cell's fields
 * (n, e, beta) and its tau (per instance, tau field, or with eta/s held the
 * rule's tau at these fields): T = e/(3n); s = 4n - n ln(n/n_eq) with
 * n_eq = d_G T^3/pi^2; eta = (4/9) gamma^2 e c_l (tau - 1/2); eta_over_s.
 * d_G > 0 (16 for gluons); while eta/s is held it must equal the d_G given
 * there.  RLB_EINVAL for kappa != 1/3 (these are e = 3P relations).
 * Asynchronous. */
rlb_status rlb_transport(rlb_solver *h, double d_G, double *T, double *s, double *eta,
                         double *eta_over_s);

/* Add the per-cell tau gradient accumulated by the reverse steps since the
 * field was set or last handed over, dL/dtau(x), to dL_dtau_cell (device
 * double [cells]) and clear the accumulator.  Contributions are added per
 * cell in step order, so the result is bitwise reproducible.  RLB_EINVAL
 * when no tau field is set.  (The per-instance dL_dtau of the reverse steps
 * is then the derivative for a uniform shift of the instance's field: the
 * sum of dL/dtau(x) over its cells.) */
rlb_status rlb_adjoint_flush_tau_field(rlb_solver *h, double *dL_dtau_cell);

/* The 16-bit storages' encoder (rlb_storage RLB_F16DEV / RLB_BF16DEV: the
 * deviations from the rest equilibrium stored as binary16 or bfloat16), on n
 * FP32 values: dst[i] is the element the step kernels store for the value
 * src[i], rounded to nearest, ties to even (bfloat16: the upper 16 bits of
 * the binary32 pattern after rounding on the discarded 16 bits; NaN stays
 * NaN; overflow gives infinity).  For callers that encode deviations
 * themselves.  storage: RLB_F16DEV or RLB_BF16DEV; src: device float [n];
 * dst: device 2-byte elements [n]; stream: a hipStream_t, NULL for the null
 * stream.  Enqueued, not synchronised; needs no solver.  RLB_EINVAL for
 * another storage, n < 0, or a NULL pointer with n > 0. */
rlb_status rlb_encode16(int32_t storage, const float *src, void *dst, int64_t n, void *stream);

/* Release the solver's own memory (not pop_a / pop_b).  Synchronises. */
rlb_status rlb_destroy(rlb_solver *h);

const char *rlb_status_string(rlb_status s);

/* Message of the last error on the calling thread ("" if none). */
const char *rlb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RLB_H */
