// Reference ("oracle") implementation of the relativistic lattice Boltzmann
// (RLB) scheme of Mendoza, Boghosian, Herrmann and Succi, "Lattice Boltzmann
// scheme for relativistic fluids" (arXiv:0912.2913).
//
// TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle_rlb.so and is
// loaded by the test-suite, by the smoke check and by the CPU-baseline leg of
// the benchmark.  The GPU library never links, includes or calls it, and it
// shares no tables, headers or helpers with the GPU code: the lattice tables
// below are written out here independently.
//
// Plain, slow, single-threaded FP64 loops.  Every routine is templated on the
// scalar so that std::complex<double> runs give complex-step derivatives
// (Im L(x + i h) / h), which the gradient checks use as an exact reference.
//
// Passages followed:
//   * D3Q19 velocity set and weights: text around Fig. 2 ("Set of discrete
//     velocities ...") and the paragraph after eq. (equil2b): w0 = 1/3,
//     w = 1/18 for |c_i| = c_l, w = 1/36 for |c_i| = sqrt(2) c_l.
//   * macroscopic constraints: n gamma = sum f_i, (e+P) gamma^2 - P = sum g_i,
//     (e+P) gamma^2 u = sum g_i c_i, closed by e = 3P (paragraph before
//     eq. (lbe1)).
//   * BGK update with one tau for both populations: eqs. (lbe1), (lbe2).
//   * ultra-relativistic equilibria: eqs. (equil1s), (equil2as), (equil2bs),
//     written literally with gamma^2 = 1/(1 - |beta|^2) and c = 1.
//   * general equation of state: eqs. (equil1), (equil2a), (equil2b) with
//     P = kappa e (kappa = 1/3 selects the ultra-relativistic forms above).
//
//   * shear viscosity of the model, eta = (4/9) gamma^2 e (tau - dt/2) c_l^2
//     (end of the equilibrium section), and the transport quantities of the
//     shock-tube section: T = e / (3n), n_eq = d_G T^3 / pi^2, fugacity
//     lambda = n / n_eq, entropy density s = 4n - n ln(lambda).
//
// Readings where the paper is silent (each one is listed in the design notes):
//   * velocity ordering (Fig. 2 is missing): 0 rest; 1..6 the axis pairs
//     (+x,-x,+y,-y,+z,-z); 7..18 the diagonal pairs (xy, xz, yz), each pair
//     being (v, -v), so that opp(2k-1) = 2k.
//   * moment inversion: the paper states the relations only.  With
//     W = (4/3) e gamma^2 they give 3 W^2 - 4 E W + |M|^2 = 0; the root that is
//     continuous with rest (W = 4E/3 at M = 0) is taken.  No clamping: NaN
//     propagates.
//   * stored state: the post-collision populations S_t; one step is
//     S_{t+1}(x) = collide(pull(S_t))(x) with tau in units of dt.
//   * boundaries (not in the paper): periodic wrap, outflow = zero-gradient copy
//     (pull source clamped into the domain per axis), inflow face held at the
//     equilibrium of a given state, half-way bounce-back off solid cells
//     (pull from a solid source returns the cell's own opposite population).
//     Precedence: wrap/clamp per axis, then the solid test on the resolved
//     source.  Solid cells are never updated and hold zeros.
//   * relaxation time: tau per instance, or a per-cell field tau(x), or (to
//     hold eta/s fixed, as the shock-tube section characterises its runs by
//     eta/s) tau set in every cell and step from its pre-collision moments by
//     solving the viscosity relation for tau with eta = (eta/s) s.  Lattice
//     units: dx = 1, dt = 1/c_l, tau in units of dt, so
//     eta = (4/9) gamma^2 e c_l (tau - 1/2).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

using cplx = std::complex<double>;

constexpr int Q = 19;

// D3Q19 integer velocities e_i (c_i = c_l e_i).
const int EV[Q][3] = {
    {0, 0, 0},                                          // rest
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

double weight(int q) {
  int s = EV[q][0] * EV[q][0] + EV[q][1] * EV[q][1] + EV[q][2] * EV[q][2];
  if (s == 0) return 1.0 / 3.0;
  if (s == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

// Opposite direction, found by search rather than from the pairing rule.
int opposite(int q) {
  for (int p = 0; p < Q; ++p)
    if (EV[p][0] == -EV[q][0] && EV[p][1] == -EV[q][1] && EV[p][2] == -EV[q][2]) return p;
  return -1;
}

inline double re(double v) { return v; }
inline double re(const cplx &v) { return v.real(); }

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_INFLOW = 2 };

struct Lattice {
  int n[3];  // extents along x, y, z
  int batch;
  double c_l;
  double kappa;  // equation of state P = kappa e
  int bc[3][2];
  long cells() const { return (long)batch * n[0] * n[1] * n[2]; }
  long index(int b, int x, int y, int z) const {
    return (((long)b * n[2] + z) * n[1] + y) * n[0] + x;
  }
  bool inflow(const int c[3]) const {
    for (int a = 0; a < 3; ++a) {
      if (bc[a][0] == BC_INFLOW && c[a] == 0) return true;
      if (bc[a][1] == BC_INFLOW && c[a] == n[a] - 1) return true;
    }
    return false;
  }
  // Resolve one coordinate of a pull source: wrap on periodic axes, clamp
  // otherwise.
  int resolve(int a, int r) const {
    if (bc[a][0] == BC_PERIODIC) return ((r % n[a]) + n[a]) % n[a];
    if (r < 0) return 0;
    if (r >= n[a]) return n[a] - 1;
    return r;
  }
};

Lattice make_lattice(const int32_t *dims, double c_l, const int32_t *bc) {
  Lattice L;
  L.n[0] = dims[0];
  L.n[1] = dims[1];
  L.n[2] = dims[2];
  L.batch = dims[3];
  L.c_l = c_l;
  L.kappa = 1.0 / 3.0;
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) L.bc[a][s] = bc[2 * a + s];
  return L;
}

// ---------------------------------------------------------------------------
// Equilibria, eqs. (equil1s), (equil2as), (equil2bs), literally, with u = beta
// (c = 1) and c_i = c_l e_i.
template <class T>
void equilibria(T n, T eps, const T beta[3], double c_l, T feq[Q], T geq[Q]) {
  using std::sqrt;
  T u2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
  T gamma2 = 1.0 / (1.0 - u2);
  T gamma = sqrt(gamma2);
  double cl2 = c_l * c_l;
  for (int q = 0; q < Q; ++q) {
    double w = weight(q);
    double c[3] = {c_l * EV[q][0], c_l * EV[q][1], c_l * EV[q][2]};
    T cu = c[0] * beta[0] + c[1] * beta[1] + c[2] * beta[2];
    feq[q] = w * n * gamma * (1.0 + 3.0 * cu / cl2);
    if (q > 0)
      geq[q] = w * eps * gamma2 *
               (1.0 / (gamma2 * cl2) + 4.0 * cu / cl2 + 6.0 * cu * cu / (cl2 * cl2) -
                2.0 * u2 / cl2);
    else
      geq[q] = w * eps * gamma2 * (4.0 - (2.0 + cl2) / (gamma2 * cl2) - 2.0 * u2 / cl2);
  }
}

// Moment sums as the macroscopic constraints define them: N = sum f_i,
// E = sum g_i, M = sum g_i c_i (summed in direction order 0..18).
template <class T>
void moment_sums(const T f[Q], const T g[Q], double c_l, T *N, T *E, T M[3]) {
  T n_ = 0.0, e_ = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
  for (int q = 0; q < Q; ++q) {
    n_ += f[q];
    e_ += g[q];
    m0 += g[q] * (c_l * EV[q][0]);
    m1 += g[q] * (c_l * EV[q][1]);
    m2 += g[q] * (c_l * EV[q][2]);
  }
  *N = n_;
  *E = e_;
  M[0] = m0;
  M[1] = m1;
  M[2] = m2;
}

// Inversion of the constraints under e = 3P.  Unknowns (n, e, beta); with
// W = (e+P) gamma^2 = (4/3) e gamma^2: E = W - e/3, M = W beta, which gives the
// quadratic 3 W^2 - 4 E W + |M|^2 = 0.  The rest-continuous root is taken, then
// beta = M / W, gamma^2 = 1/(1-|beta|^2), e = 3 W / (4 gamma^2), n = N / gamma.
// Returns false when the state is unphysical (negative discriminant, e <= 0,
// |beta| >= 1, or NaN).
template <class T>
bool invert(T N, T E, const T M[3], T *n, T *eps, T beta[3]) {
  using std::sqrt;
  T M2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  T disc = 4.0 * E * E - 3.0 * M2;
  T W = (2.0 * E + sqrt(disc)) / 3.0;
  for (int a = 0; a < 3; ++a) beta[a] = M[a] / W;
  T b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
  T gamma2 = 1.0 / (1.0 - b2);
  *eps = 3.0 * W / (4.0 * gamma2);
  *n = N / sqrt(gamma2);
  bool ok = re(disc) > 0.0 && re(*eps) > 0.0 && re(b2) < 1.0;
  return ok;
}

// General-EoS equilibria, eqs. (equil1), (equil2a), (equil2b), literally, with
// the pressure P given alongside e.
template <class T>
void equilibria_eos(T n, T eps, T P, const T beta[3], double c_l, T feq[Q], T geq[Q]) {
  using std::sqrt;
  T u2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
  T gamma2 = 1.0 / (1.0 - u2);
  T gamma = sqrt(gamma2);
  double cl2 = c_l * c_l;
  for (int q = 0; q < Q; ++q) {
    double w = weight(q);
    double c[3] = {c_l * EV[q][0], c_l * EV[q][1], c_l * EV[q][2]};
    T cu = c[0] * beta[0] + c[1] * beta[1] + c[2] * beta[2];
    feq[q] = w * n * gamma * (1.0 + 3.0 * cu / cl2);
    if (q > 0)
      geq[q] = w * (eps + P) * gamma2 *
               (3.0 * P / ((P + eps) * gamma2 * cl2) + 3.0 * cu / cl2 +
                4.5 * cu * cu / (cl2 * cl2) - 1.5 * u2 / cl2);
    else
      geq[q] = w * (eps + P) * gamma2 *
               (3.0 - 3.0 * P * (2.0 + cl2) / ((P + eps) * gamma2 * cl2) - 1.5 * u2 / cl2);
  }
}

// Inversion of the constraints for P = kappa e.  With W = (e+P) gamma^2 the
// constraints read E = W - P, M = W beta, and |beta|^2 = 1 - 1/gamma^2 gives
// W^2 - (1 + kappa) E W + kappa |M|^2 = 0; the root continuous with rest
// (W = (1 + kappa) E at M = 0) is taken, then beta = M / W,
// e = W / ((1 + kappa) gamma^2), n = N / gamma.
template <class T>
bool invert_eos(T N, T E, const T M[3], double kappa, T *n, T *eps, T beta[3]) {
  using std::sqrt;
  T M2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  T disc = (1.0 + kappa) * (1.0 + kappa) * E * E - 4.0 * kappa * M2;
  T W = ((1.0 + kappa) * E + sqrt(disc)) / 2.0;
  for (int a = 0; a < 3; ++a) beta[a] = M[a] / W;
  T b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
  T gamma2 = 1.0 / (1.0 - b2);
  *eps = W / ((1.0 + kappa) * gamma2);
  *n = N / sqrt(gamma2);
  return re(disc) > 0.0 && re(*eps) > 0.0 && re(b2) < 1.0;
}

// Dispatch on the equation of state: kappa = 1/3 takes the ultra-relativistic
// forms (equil1s/equil2as/equil2bs and the e = 3P inversion), any other kappa
// the general ones.
inline bool radiation(double kappa) { return kappa == 1.0 / 3.0; }

template <class T>
void eq_any(T n, T eps, const T beta[3], double c_l, double kappa, T feq[Q], T geq[Q]) {
  if (radiation(kappa))
    equilibria(n, eps, beta, c_l, feq, geq);
  else
    equilibria_eos(n, eps, T(kappa * eps), beta, c_l, feq, geq);
}

template <class T>
bool inv_any(T N, T E, const T M[3], double kappa, T *n, T *eps, T beta[3]) {
  if (radiation(kappa)) return invert(N, E, M, n, eps, beta);
  return invert_eos(N, E, M, kappa, n, eps, beta);
}

// One BGK collision, eqs. (lbe1)/(lbe2): post = pre - (dt/tau)(pre - eq), with
// tau given in units of dt.  With do_f false the f population is skipped (its
// outputs are left untouched): f never enters (e, beta).
template <class T>
bool collide(const T pf[Q], const T pg[Q], T tau, double c_l, bool do_f, T of[Q], T og[Q],
             double kappa = 1.0 / 3.0) {
  T N, E, M[3];
  T zero[Q];
  for (int q = 0; q < Q; ++q) zero[q] = 0.0;
  moment_sums(do_f ? pf : zero, pg, c_l, &N, &E, M);
  T n, eps, beta[3];
  bool ok = inv_any(N, E, M, kappa, &n, &eps, beta);
  T feq[Q], geq[Q];
  eq_any(n, eps, beta, c_l, kappa, feq, geq);
  for (int q = 0; q < Q; ++q) {
    og[q] = pg[q] - (1.0 / tau) * (pg[q] - geq[q]);
    if (do_f) of[q] = pf[q] - (1.0 / tau) * (pf[q] - feq[q]);
  }
  return ok;
}

// Transport quantities of one cell from its fields (n, e, beta) and tau:
// temperature T = e/(3n), equilibrium density n_eq = d_G T^3/pi^2, fugacity
// lambda = n/n_eq, entropy density s = 4n - n ln(lambda), shear viscosity
// eta = (4/9) gamma^2 e (tau - dt/2) c_l^2 with dt = 1/c_l.
template <class T>
void transport(T n, T eps, const T beta[3], T tau, double c_l, double d_G, T *temp, T *s, T *eta) {
  using std::log;
  const double pi = 3.14159265358979323846;
  T Tm = eps / (3.0 * n);
  T n_eq = d_G * Tm * Tm * Tm / (pi * pi);
  T lam = n / n_eq;
  T b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
  T gamma2 = 1.0 / (1.0 - b2);
  double dt = 1.0 / c_l;
  *temp = Tm;
  *s = 4.0 * n - n * log(lam);
  *eta = (4.0 / 9.0) * gamma2 * eps * (tau * dt - dt / 2.0) * (c_l * c_l);
}

// The relaxation time that gives eta/s = eta_s at the pre-collision moments
// of one cell (both populations): the viscosity relation
// eta = (4/9) gamma^2 e (tau dt - dt/2) c_l^2 solved for tau, with
// eta = eta_s * s and s from the same moments.
template <class T>
T tau_for_eta_s(const T pf[Q], const T pg[Q], double c_l, double eta_s, double d_G) {
  T N, E, M[3], n, eps, beta[3];
  moment_sums(pf, pg, c_l, &N, &E, M);
  invert(N, E, M, &n, &eps, beta);
  T Tm, s, eta_unused;
  transport(n, eps, beta, T(1.0), c_l, d_G, &Tm, &s, &eta_unused);
  T b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
  T gamma2 = 1.0 / (1.0 - b2);
  double dt = 1.0 / c_l;
  T eta = eta_s * s;
  return (eta / ((4.0 / 9.0) * gamma2 * eps * (c_l * c_l)) + dt / 2.0) / dt;
}

// Relaxation time of every update: per instance (tau[batch]), or a per-cell
// field (tau_cell[cells]), or set from the local state to hold eta/s fixed
// (eta_s > 0, f+g steps only).
template <class T>
struct Relax {
  const T *tau;
  const T *tau_cell;
  double eta_s;
  double d_G;
};

// Where the pull of direction q at cell c comes from: (source cell index,
// source direction).  A solid resolved source means half-way bounce-back: the
// cell's own opposite population.
struct Source {
  long idx;
  int q;
};

Source pull_source(const Lattice &L, const uint8_t *solid, int b, const int c[3], int q) {
  int s[3];
  for (int a = 0; a < 3; ++a) s[a] = L.resolve(a, c[a] - EV[q][a]);
  long si = L.index(b, s[0], s[1], s[2]);
  if (solid && solid[si]) return {L.index(b, c[0], c[1], c[2]), opposite(q)};
  return {si, q};
}

// Positivity of f^eq (discussion section): every f^eq_i = w_i n gamma
// (1 + 3 c_i.u / c_l^2) is positive only while c_i.u > -c_l^2/3 for every i.
// Returns false when some direction breaks that bound (or u is NaN).
bool feq_positive(const double beta[3], double c_l) {
  const double cl2 = c_l * c_l;
  for (int q = 0; q < Q; ++q) {
    const double cu = c_l * EV[q][0] * beta[0] + c_l * EV[q][1] * beta[1] + c_l * EV[q][2] * beta[2];
    if (!(1.0 + 3.0 * cu / cl2 > 0.0)) return false;
  }
  return true;
}

// Optional record of a run's f-positivity: `lost` counts the updates whose
// f^eq broke the bound above; per cell, `mark` is set once the cell's f has
// depended on such an update (the update itself, or a pull from a marked
// source: the loss travels with the populations, bounce-back included).
// Held cells (inflow, solid) are never marked.
struct PosTrack {
  std::vector<uint8_t> mark, next;
  long lost = 0;
};

// One full time step S_in -> S_out.  Layout S[pop][q][cell], pop 0 = f, 1 = g
// (cells = batch * nz * ny * nx, x fastest).  With do_f false only the g block
// is read and written (the pointers then address a g block of 19*cells).
// trk (f+g FP64 runs only) records f-positivity.
template <class T>
long step(const Lattice &L, const Relax<T> &rx, const uint8_t *solid, const T in_f[Q],
          const T in_g[Q], const T *Sin, T *Sout, bool do_f, PosTrack *trk = nullptr) {
  const long C = L.cells();
  const T *fin = Sin, *gin = do_f ? Sin + (long)Q * C : Sin;
  T *fout = Sout, *gout = do_f ? Sout + (long)Q * C : Sout;
  long unphysical = 0;
  for (int b = 0; b < L.batch; ++b)
    for (int z = 0; z < L.n[2]; ++z)
      for (int y = 0; y < L.n[1]; ++y)
        for (int x = 0; x < L.n[0]; ++x) {
          int c[3] = {x, y, z};
          long i = L.index(b, x, y, z);
          if (solid && solid[i]) {
            for (int q = 0; q < Q; ++q) {
              gout[(long)q * C + i] = 0.0;
              if (do_f) fout[(long)q * C + i] = 0.0;
            }
            if (trk) trk->next[i] = 0;
            continue;
          }
          if (L.inflow(c)) {
            for (int q = 0; q < Q; ++q) {
              gout[(long)q * C + i] = in_g[q];
              if (do_f) fout[(long)q * C + i] = in_f[q];
            }
            if (trk) trk->next[i] = 0;
            continue;
          }
          T pf[Q], pg[Q], of[Q], og[Q];
          bool marked = false;
          for (int q = 0; q < Q; ++q) {
            Source s = pull_source(L, solid, b, c, q);
            pg[q] = gin[(long)s.q * C + s.idx];
            pf[q] = do_f ? fin[(long)s.q * C + s.idx] : T(0.0);
            if (trk && trk->mark[s.idx]) marked = true;
          }
          T tau = rx.tau_cell ? rx.tau_cell[i] : rx.tau[b];
          if (rx.eta_s > 0.0) tau = tau_for_eta_s(pf, pg, L.c_l, rx.eta_s, rx.d_G);
          if (!collide(pf, pg, tau, L.c_l, do_f, of, og, L.kappa)) ++unphysical;
          if (trk) {
            // u of this update, as the collision obtained it
            T N, E, M[3], n, eps, beta[3];
            moment_sums(pf, pg, L.c_l, &N, &E, M);
            inv_any(N, E, M, L.kappa, &n, &eps, beta);
            const double u[3] = {re(beta[0]), re(beta[1]), re(beta[2])};
            if (!feq_positive(u, L.c_l)) {
              ++trk->lost;
              marked = true;
            }
            trk->next[i] = marked ? 1 : 0;
          }
          for (int q = 0; q < Q; ++q) {
            gout[(long)q * C + i] = og[q];
            if (do_f) fout[(long)q * C + i] = of[q];
          }
        }
  if (trk) std::swap(trk->mark, trk->next);
  return unphysical;
}

template <class T>
void inflow_equilibria(const Lattice &L, T in_n, T in_e, const T in_b[3], T in_f[Q], T in_g[Q]) {
  eq_any(in_n, in_e, in_b, L.c_l, L.kappa, in_f, in_g);
}

// S_0: equilibrium of the initial fields; inflow cells take the inflow state;
// solid cells hold zeros.  beta0 is [3][cells].
template <class T>
void init_state(const Lattice &L, const uint8_t *solid, const T *n0, const T *e0, const T *beta0,
                const T in_f[Q], const T in_g[Q], T *S, bool do_f) {
  const long C = L.cells();
  T *f = S, *g = do_f ? S + (long)Q * C : S;
  for (int b = 0; b < L.batch; ++b)
    for (int z = 0; z < L.n[2]; ++z)
      for (int y = 0; y < L.n[1]; ++y)
        for (int x = 0; x < L.n[0]; ++x) {
          int c[3] = {x, y, z};
          long i = L.index(b, x, y, z);
          T feq[Q], geq[Q];
          if (solid && solid[i]) {
            for (int q = 0; q < Q; ++q) feq[q] = geq[q] = 0.0;
          } else if (L.inflow(c)) {
            for (int q = 0; q < Q; ++q) {
              feq[q] = in_f[q];
              geq[q] = in_g[q];
            }
          } else {
            T beta[3] = {beta0[i], beta0[C + i], beta0[2 * C + i]};
            T n = do_f ? n0[i] : T(1.0);
            eq_any(n, e0[i], beta, L.c_l, L.kappa, feq, geq);
          }
          for (int q = 0; q < Q; ++q) {
            g[(long)q * C + i] = geq[q];
            if (do_f) f[(long)q * C + i] = feq[q];
          }
        }
}

// Fields of a stored state: (n, e, beta) per cell (zeros on solid cells).
template <class T>
void fields(const Lattice &L, const uint8_t *solid, const T *S, bool do_f, T *n, T *e, T *beta) {
  const long C = L.cells();
  const T *f = S, *g = do_f ? S + (long)Q * C : S;
  for (long i = 0; i < C; ++i) {
    if (solid && solid[i]) {
      if (n) n[i] = 0.0;
      e[i] = 0.0;
      beta[i] = beta[C + i] = beta[2 * C + i] = 0.0;
      continue;
    }
    T pf[Q], pg[Q];
    for (int q = 0; q < Q; ++q) {
      pg[q] = g[(long)q * C + i];
      pf[q] = do_f ? f[(long)q * C + i] : T(0.0);
    }
    T N, E, M[3], nn, ee, bb[3];
    moment_sums(pf, pg, L.c_l, &N, &E, M);
    inv_any(N, E, M, L.kappa, &nn, &ee, bb);
    if (n) n[i] = nn;
    e[i] = ee;
    beta[i] = bb[0];
    beta[C + i] = bb[1];
    beta[2 * C + i] = bb[2];
  }
}

// Loss on the final fields, over non-solid cells:
//   L = sum_x a(x) (e(x) - t(x))^2 + sum_x be(x) e(x) + sum_x sum_k bb_k(x) beta_k(x)
// Any of a/t, be, bb may be null.
struct LossSpec {
  const double *a, *t, *be, *bb;
};

template <class T>
T loss_value(const Lattice &L, const uint8_t *solid, const T *e, const T *beta, const LossSpec &ls) {
  const long C = L.cells();
  T acc = 0.0;
  for (long i = 0; i < C; ++i) {
    if (solid && solid[i]) continue;
    if (ls.a) {
      T d = e[i] - ls.t[i];
      acc += ls.a[i] * d * d;
    }
    if (ls.be) acc += ls.be[i] * e[i];
    if (ls.bb)
      for (int k = 0; k < 3; ++k) acc += ls.bb[k * C + i] * beta[k * C + i];
  }
  return acc;
}

// Complex-step derivative of the g-collision output with respect to every
// input of one cell: J[q][p] = d post_q / d pre_p, and d post_q / d tau.
void collide_jacobian(const double pg[Q], double tau, double c_l, double kappa, double J[Q][Q],
                      double dtau[Q]) {
  const double h = 1e-30;
  cplx zf[Q], of[Q], og[Q], cg[Q];
  for (int q = 0; q < Q; ++q) zf[q] = 0.0;
  for (int p = 0; p < Q; ++p) {
    for (int q = 0; q < Q; ++q) cg[q] = cplx(pg[q], q == p ? h : 0.0);
    collide<cplx>(zf, cg, cplx(tau, 0.0), c_l, false, of, og, kappa);
    for (int q = 0; q < Q; ++q) J[q][p] = og[q].imag() / h;
  }
  for (int q = 0; q < Q; ++q) cg[q] = cplx(pg[q], 0.0);
  collide<cplx>(zf, cg, cplx(tau, h), c_l, false, of, og, kappa);
  for (int q = 0; q < Q; ++q) dtau[q] = og[q].imag() / h;
}

// d g^eq_q / d(e, beta_0, beta_1, beta_2) at (e, beta) by complex step.
void geq_jacobian(double e, const double beta[3], double c_l, double kappa, double J[Q][4]) {
  const double h = 1e-30;
  cplx feq[Q], geq[Q];
  for (int k = 0; k < 4; ++k) {
    cplx ce(e, k == 0 ? h : 0.0);
    cplx cb[3] = {cplx(beta[0], k == 1 ? h : 0.0), cplx(beta[1], k == 2 ? h : 0.0),
                  cplx(beta[2], k == 3 ? h : 0.0)};
    eq_any<cplx>(cplx(1.0, 0.0), ce, cb, c_l, kappa, feq, geq);
    for (int q = 0; q < Q; ++q) J[q][k] = geq[q].imag() / h;
  }
}

// d(e, beta_0, beta_1, beta_2) / d g_p of one stored cell, by complex step on
// the moment inversion.
void fields_jacobian(const double g[Q], double c_l, double kappa, double J[4][Q]) {
  const double h = 1e-30;
  cplx cf[Q], cg[Q];
  for (int q = 0; q < Q; ++q) cf[q] = 0.0;
  for (int p = 0; p < Q; ++p) {
    for (int q = 0; q < Q; ++q) cg[q] = cplx(g[q], q == p ? h : 0.0);
    cplx N, E, M[3], n, e, b[3];
    moment_sums(cf, cg, c_l, &N, &E, M);
    inv_any(N, E, M, kappa, &n, &e, b);
    J[0][p] = e.imag() / h;
    for (int k = 0; k < 3; ++k) J[1 + k][p] = b[k].imag() / h;
  }
}

// One reverse step of the g population: lam_t = (d S_{t+1} / d S_t)^T lam_{t+1},
// built literally as the transpose of the pull map: every updated cell forms
// mu = J^T lam_{t+1}(x) from its complex-step collision Jacobian and adds each
// mu_p to the stored population it pulled from.  Inflow cells (held at the
// inflow equilibrium) route lam_{t+1} into d/d(e_in, beta_in); tau adds
// lam . d post / d tau.
void adjoint_step_g(const Lattice &L, const Relax<double> &rx, const uint8_t *solid, double in_e,
                    const double in_b[3], const double *Sg, const double *lam_next,
                    double *lam_out, double *dtau, double *dbeta_in, double *de_in,
                    double *dtau_cell) {
  const long C = L.cells();
  for (long k = 0; k < (long)Q * C; ++k) lam_out[k] = 0.0;
  double Jin[Q][4];
  geq_jacobian(in_e, in_b, L.c_l, L.kappa, Jin);
  for (int b = 0; b < L.batch; ++b)
    for (int z = 0; z < L.n[2]; ++z)
      for (int y = 0; y < L.n[1]; ++y)
        for (int x = 0; x < L.n[0]; ++x) {
          int c[3] = {x, y, z};
          long i = L.index(b, x, y, z);
          if (solid && solid[i]) continue;
          double lam[Q];
          for (int q = 0; q < Q; ++q) lam[q] = lam_next[(long)q * C + i];
          if (L.inflow(c)) {
            for (int q = 0; q < Q; ++q) {
              if (de_in) *de_in += lam[q] * Jin[q][0];
              if (dbeta_in)
                for (int k = 0; k < 3; ++k) dbeta_in[k] += lam[q] * Jin[q][1 + k];
            }
            continue;
          }
          double pg[Q];
          Source src[Q];
          for (int q = 0; q < Q; ++q) {
            src[q] = pull_source(L, solid, b, c, q);
            pg[q] = Sg[(long)src[q].q * C + src[q].idx];
          }
          double J[Q][Q], dt[Q];
          collide_jacobian(pg, rx.tau_cell ? rx.tau_cell[i] : rx.tau[b], L.c_l, L.kappa, J, dt);
          for (int p = 0; p < Q; ++p) {
            double mu = 0.0;
            for (int q = 0; q < Q; ++q) mu += lam[q] * J[q][p];
            lam_out[(long)src[p].q * C + src[p].idx] += mu;
          }
          if (dtau || dtau_cell) {
            double s = 0.0;
            for (int q = 0; q < Q; ++q) s += lam[q] * dt[q];
            if (dtau) dtau[b] += s;
            if (dtau_cell) dtau_cell[i] += s;
          }
        }
}

// lam_T = (d(e, beta)/d S_T)^T (dL/de, dL/dbeta) per non-solid cell.
void moments_adjoint_g(const Lattice &L, const uint8_t *solid, const double *Sg, const double *dLde,
                       const double *dLdb, double *lam) {
  const long C = L.cells();
  for (long i = 0; i < C; ++i) {
    if (solid && solid[i]) {
      for (int q = 0; q < Q; ++q) lam[(long)q * C + i] = 0.0;
      continue;
    }
    double g[Q], J[4][Q];
    for (int q = 0; q < Q; ++q) g[q] = Sg[(long)q * C + i];
    fields_jacobian(g, L.c_l, L.kappa, J);
    for (int p = 0; p < Q; ++p) {
      double v = dLde[i] * J[0][p];
      for (int k = 0; k < 3; ++k) v += dLdb[k * C + i] * J[1 + k][p];
      lam[(long)p * C + i] = v;
    }
  }
}

// Initial state S_0 = g^eq(e0, beta0) on interior cells, g^eq(e_in, beta_in) on
// inflow cells: lam_0 -> dL/de0, dL/dbeta0 (+= into the inflow gradients).
void init_adjoint_g(const Lattice &L, const uint8_t *solid, const double *e0, const double *beta0,
                    double in_e, const double in_b[3], const double *lam, double *dLde0,
                    double *dLdb0, double *dbeta_in, double *de_in) {
  const long C = L.cells();
  double Jin[Q][4];
  geq_jacobian(in_e, in_b, L.c_l, L.kappa, Jin);
  for (int b = 0; b < L.batch; ++b)
    for (int z = 0; z < L.n[2]; ++z)
      for (int y = 0; y < L.n[1]; ++y)
        for (int x = 0; x < L.n[0]; ++x) {
          int c[3] = {x, y, z};
          long i = L.index(b, x, y, z);
          dLde0[i] = 0.0;
          dLdb0[i] = dLdb0[C + i] = dLdb0[2 * C + i] = 0.0;
          if (solid && solid[i]) continue;
          if (L.inflow(c)) {
            for (int q = 0; q < Q; ++q) {
              double l = lam[(long)q * C + i];
              if (de_in) *de_in += l * Jin[q][0];
              if (dbeta_in)
                for (int k = 0; k < 3; ++k) dbeta_in[k] += l * Jin[q][1 + k];
            }
            continue;
          }
          double bt[3] = {beta0[i], beta0[C + i], beta0[2 * C + i]};
          double J[Q][4];
          geq_jacobian(e0[i], bt, L.c_l, L.kappa, J);
          double s[4] = {0, 0, 0, 0};
          for (int q = 0; q < Q; ++q) {
            double l = lam[(long)q * C + i];
            for (int k = 0; k < 4; ++k) s[k] += l * J[q][k];
          }
          dLde0[i] = s[0];
          for (int k = 0; k < 3; ++k) dLdb0[k * C + i] = s[1 + k];
        }
}

Relax<double> relax_of(const void *r);

}  // namespace

// ===========================================================================
// C entry points (ctypes).  Arrays are host arrays in the oracle layout:
// populations [2][19][cells] (or [19][cells] for g-only calls), fields [cells],
// beta [3][cells], with cells = batch*nz*ny*nx, x fastest.  dims = {nx, ny, nz,
// batch}; bc = {x_lo, x_hi, y_lo, y_hi, z_lo, z_hi} (0 periodic, 1 outflow,
// 2 inflow); inflow = {n, e, beta_x, beta_y, beta_z}.
extern "C" {

// Parameters of a run: tau[batch]; optional tau_cell[cells]; eta_s > 0 holds
// eta/s fixed with degeneracy d_G (f+g runs only); kappa: P = kappa e
// (0 means 1/3, the paper's e = 3P).
struct OraRelax {
  const double *tau;
  const double *tau_cell;
  double eta_s;
  double d_G;
  double kappa;
};

static double kappa_of(double k) { return k == 0.0 ? 1.0 / 3.0 : k; }

int ora_num_directions() { return Q; }

void ora_lattice(int32_t *e /*[19][3]*/, double *w /*[19]*/, int32_t *opp /*[19]*/) {
  for (int q = 0; q < Q; ++q) {
    for (int a = 0; a < 3; ++a) e[3 * q + a] = EV[q][a];
    w[q] = weight(q);
    opp[q] = opposite(q);
  }
}

void ora_equilibria(double n, double eps, const double *beta, double c_l, double kappa,
                    double *feq, double *geq) {
  eq_any<double>(n, eps, beta, c_l, kappa_of(kappa), feq, geq);
}

int ora_invert(double N, double E, const double *M, double kappa,
               double *out /* n, e, bx, by, bz */) {
  double n, e, b[3];
  bool ok = inv_any<double>(N, E, M, kappa_of(kappa), &n, &e, b);
  out[0] = n;
  out[1] = e;
  out[2] = b[0];
  out[3] = b[1];
  out[4] = b[2];
  return ok ? 1 : 0;
}

int ora_collide(const double *pf, const double *pg, double tau, double c_l, double kappa,
                double *of, double *og) {
  return collide<double>(pf, pg, tau, c_l, true, of, og, kappa_of(kappa)) ? 1 : 0;
}

void ora_init(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
              const uint8_t *solid, double kappa, const double *n0, const double *e0,
              const double *beta0, double *S) {
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(kappa);
  double in_f[Q], in_g[Q];
  inflow_equilibria<double>(L, inflow[0], inflow[1], inflow + 2, in_f, in_g);
  init_state<double>(L, solid, n0, e0, beta0, in_f, in_g, S, true);
}

// Runs nsteps f+g steps in place on S (a scratch copy is allocated here).
// Returns the number of unphysical cell updates seen.
long ora_run(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
             const uint8_t *solid, const OraRelax *rxp, double *S, int nsteps) {
  const Relax<double> rx = relax_of(rxp);
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  if (rx.eta_s > 0.0 && !radiation(L.kappa)) return -1;  // the eta/s rule is for e = 3P
  double in_f[Q], in_g[Q];
  inflow_equilibria<double>(L, inflow[0], inflow[1], inflow + 2, in_f, in_g);
  const long n = 2L * Q * L.cells();
  std::vector<double> tmp(n);
  double *a = S, *b = tmp.data();
  long bad = 0;
  for (int t = 0; t < nsteps; ++t) {
    bad += step<double>(L, rx, solid, in_f, in_g, a, b, true);
    std::swap(a, b);
  }
  if (a != S) std::memcpy(S, a, n * sizeof(double));
  return bad;
}

// ora_run with a record of f-positivity (see PosTrack): *lost = updates whose
// f^eq broke the bound c_i.u > -c_l^2/3; mark[cells] = 1 where the final f
// depends on such an update.  mark may hold an earlier run's record (it is
// carried on), or zeros.
long ora_run_tracked(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
                     const uint8_t *solid, const OraRelax *rxp, double *S, int nsteps,
                     uint8_t *mark, long *lost) {
  const Relax<double> rx = relax_of(rxp);
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  if (rx.eta_s > 0.0 && !radiation(L.kappa)) return -1;
  double in_f[Q], in_g[Q];
  inflow_equilibria<double>(L, inflow[0], inflow[1], inflow + 2, in_f, in_g);
  const long C = L.cells();
  const long n = 2L * Q * C;
  std::vector<double> tmp(n);
  PosTrack trk;
  trk.mark.assign(mark, mark + C);
  trk.next.assign(C, 0);
  double *a = S, *b = tmp.data();
  long bad = 0;
  for (int t = 0; t < nsteps; ++t) {
    bad += step<double>(L, rx, solid, in_f, in_g, a, b, true, &trk);
    std::swap(a, b);
  }
  if (a != S) std::memcpy(S, a, n * sizeof(double));
  std::memcpy(mark, trk.mark.data(), C);
  *lost = trk.lost;
  return bad;
}

// Same as ora_run on the g population only (S is [19][cells]).
long ora_run_g(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
               const uint8_t *solid, const OraRelax *rxp, double *S, int nsteps) {
  const Relax<double> rx = relax_of(rxp);
  if (rx.eta_s > 0.0) return -1;  // holding eta/s needs n, i.e. the f population
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  double in_f[Q], in_g[Q];
  inflow_equilibria<double>(L, inflow[0], inflow[1], inflow + 2, in_f, in_g);
  const long n = (long)Q * L.cells();
  std::vector<double> tmp(n);
  double *a = S, *b = tmp.data();
  long bad = 0;
  for (int t = 0; t < nsteps; ++t) {
    bad += step<double>(L, rx, solid, in_f, in_g, a, b, false);
    std::swap(a, b);
  }
  if (a != S) std::memcpy(S, a, n * sizeof(double));
  return bad;
}

// Post-step populations of selected cells only: out[k][0..37] = (f_0..f_18,
// g_0..g_18) of cell idx[k] after one step from S (the full stored state).
void ora_update_cells(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
                      const uint8_t *solid, const OraRelax *rxp, const double *S, long ncells,
                      const long *idx, double *out) {
  const Relax<double> rx = relax_of(rxp);
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  double in_f[Q], in_g[Q];
  inflow_equilibria<double>(L, inflow[0], inflow[1], inflow + 2, in_f, in_g);
  const long C = L.cells();
  const double *f = S, *g = S + (long)Q * C;
  for (long k = 0; k < ncells; ++k) {
    long i = idx[k];
    long r = i;
    int c[3];
    c[0] = (int)(r % L.n[0]);
    r /= L.n[0];
    c[1] = (int)(r % L.n[1]);
    r /= L.n[1];
    c[2] = (int)(r % L.n[2]);
    int b = (int)(r / L.n[2]);
    double *o = out + 2 * Q * k;
    if (solid && solid[i]) {
      for (int q = 0; q < 2 * Q; ++q) o[q] = 0.0;
      continue;
    }
    if (L.inflow(c)) {
      for (int q = 0; q < Q; ++q) {
        o[q] = in_f[q];
        o[Q + q] = in_g[q];
      }
      continue;
    }
    double pf[Q], pg[Q];
    for (int q = 0; q < Q; ++q) {
      Source s = pull_source(L, solid, b, c, q);
      pf[q] = f[(long)s.q * C + s.idx];
      pg[q] = g[(long)s.q * C + s.idx];
    }
    double tau = rx.tau_cell ? rx.tau_cell[i] : rx.tau[b];
    if (rx.eta_s > 0.0) tau = tau_for_eta_s(pf, pg, L.c_l, rx.eta_s, rx.d_G);
    collide<double>(pf, pg, tau, L.c_l, true, o, o + Q, L.kappa);
  }
}

// Fields (n, e, beta[3][cells]) and per-instance conservation sums
// sums[b][5] = (sum f, sum g, sum g c_x, sum g c_y, sum g c_z) over non-solid
// cells.
void ora_moments(const int32_t *dims, double c_l, double kappa, const uint8_t *solid,
                 const double *S, double *n, double *e, double *beta, double *sums) {
  int32_t bc0[6] = {0, 0, 0, 0, 0, 0};
  Lattice L = make_lattice(dims, c_l, bc0);
  L.kappa = kappa_of(kappa);
  fields<double>(L, solid, S, true, n, e, beta);
  if (!sums) return;
  const long C = L.cells();
  const long per = (long)L.n[0] * L.n[1] * L.n[2];
  for (int b = 0; b < L.batch; ++b) {
    double s[5] = {0, 0, 0, 0, 0};
    for (long j = 0; j < per; ++j) {
      long i = b * per + j;
      if (solid && solid[i]) continue;
      for (int q = 0; q < Q; ++q) {
        double fv = S[(long)q * C + i], gv = S[(long)(Q + q) * C + i];
        s[0] += fv;
        s[1] += gv;
        for (int a = 0; a < 3; ++a) s[2 + a] += gv * (c_l * EV[q][a]);
      }
    }
    for (int k = 0; k < 5; ++k) sums[5 * b + k] = s[k];
  }
}

// g-only versions of the reverse-mode building blocks (oracle layout
// [19][cells]); gradients are accumulated (+=) except lam_out / lam / dLde0 /
// dLdb0 which are overwritten.
int ora_adjoint_step(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
                     const uint8_t *solid, const OraRelax *rxp, const double *Sg,
                     const double *lam_next, double *lam_out, double *dtau, double *dbeta_in,
                     double *de_in, double *dtau_cell) {
  const Relax<double> rx = relax_of(rxp);
  if (rx.eta_s > 0.0) return 0;  // g-only reverse mode does not hold with tau(n)
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  adjoint_step_g(L, rx, solid, inflow[1], inflow + 2, Sg, lam_next, lam_out, dtau, dbeta_in,
                 de_in, dtau_cell);
  return 1;
}

void ora_moments_adjoint(const int32_t *dims, double c_l, double kappa, const uint8_t *solid,
                         const double *Sg, const double *dLde, const double *dLdb, double *lam) {
  int32_t bc0[6] = {0, 0, 0, 0, 0, 0};
  Lattice L = make_lattice(dims, c_l, bc0);
  L.kappa = kappa_of(kappa);
  moments_adjoint_g(L, solid, Sg, dLde, dLdb, lam);
}

void ora_init_adjoint(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
                      const uint8_t *solid, double kappa, const double *e0, const double *beta0,
                      const double *lam, double *dLde0, double *dLdb0, double *dbeta_in,
                      double *de_in) {
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(kappa);
  init_adjoint_g(L, solid, e0, beta0, inflow[1], inflow + 2, lam, dLde0, dLdb0, dbeta_in, de_in);
}

// Loss of a g-only forward run of nsteps from the initial fields (FP64).
double ora_loss(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
                const uint8_t *solid, const OraRelax *rxp, const double *e0, const double *beta0,
                int nsteps, const double *la, const double *lt, const double *lbe,
                const double *lbb) {
  const Relax<double> rx = relax_of(rxp);
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  const long C = L.cells();
  double in_f[Q], in_g[Q];
  inflow_equilibria<double>(L, inflow[0], inflow[1], inflow + 2, in_f, in_g);
  std::vector<double> a((long)Q * C), b((long)Q * C);
  init_state<double>(L, solid, nullptr, e0, beta0, in_f, in_g, a.data(), false);
  double *p = a.data(), *q = b.data();
  for (int t = 0; t < nsteps; ++t) {
    step<double>(L, rx, solid, in_f, in_g, p, q, false);
    std::swap(p, q);
  }
  std::vector<double> e(C), bt(3 * C);
  fields<double>(L, solid, p, false, nullptr, e.data(), bt.data());
  LossSpec ls{la, lt, lbe, lbb};
  return loss_value<double>(L, solid, e.data(), bt.data(), ls);
}

// Complex-step directional derivative of the same loss: every parameter is
// perturbed by i*h times its direction (d_tau[batch], d_inflow = {d e_in,
// d beta_in[3]}, d_e0[cells], d_beta0[3][cells]; any may be null = zero).
// Returns dL . d (and the loss itself in *loss).
double ora_loss_cs(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
                   const uint8_t *solid, const OraRelax *rxp, const double *e0,
                   const double *beta0, int nsteps, const double *la, const double *lt,
                   const double *lbe, const double *lbb, const double *d_tau,
                   const double *d_inflow, const double *d_e0, const double *d_beta0,
                   const double *d_tau_cell, double *loss) {
  const double h = 1e-30;
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  const long C = L.cells();
  const double *tau = rxp->tau;
  std::vector<cplx> ctau(L.batch), ce0(C), cb0(3 * C), ctc;
  for (int b = 0; b < L.batch; ++b) ctau[b] = cplx(tau[b], d_tau ? h * d_tau[b] : 0.0);
  if (rxp->tau_cell) {
    ctc.resize(C);
    for (long i = 0; i < C; ++i)
      ctc[i] = cplx(rxp->tau_cell[i], d_tau_cell ? h * d_tau_cell[i] : 0.0);
  }
  const Relax<cplx> crx{ctau.data(), rxp->tau_cell ? ctc.data() : nullptr, 0.0, rxp->d_G};
  for (long i = 0; i < C; ++i) ce0[i] = cplx(e0[i], d_e0 ? h * d_e0[i] : 0.0);
  for (long i = 0; i < 3 * C; ++i) cb0[i] = cplx(beta0[i], d_beta0 ? h * d_beta0[i] : 0.0);
  cplx in_n(inflow[0], 0.0), in_e(inflow[1], d_inflow ? h * d_inflow[0] : 0.0);
  cplx in_b[3];
  for (int k = 0; k < 3; ++k) in_b[k] = cplx(inflow[2 + k], d_inflow ? h * d_inflow[1 + k] : 0.0);
  cplx in_f[Q], in_g[Q];
  inflow_equilibria<cplx>(L, in_n, in_e, in_b, in_f, in_g);
  std::vector<cplx> a((long)Q * C), b((long)Q * C);
  init_state<cplx>(L, solid, nullptr, ce0.data(), cb0.data(), in_f, in_g, a.data(), false);
  cplx *p = a.data(), *q = b.data();
  for (int t = 0; t < nsteps; ++t) {
    step<cplx>(L, crx, solid, in_f, in_g, p, q, false);
    std::swap(p, q);
  }
  std::vector<cplx> e(C), bt(3 * C);
  fields<cplx>(L, solid, p, false, nullptr, e.data(), bt.data());
  LossSpec ls{la, lt, lbe, lbb};
  cplx Lc = loss_value<cplx>(L, solid, e.data(), bt.data(), ls);
  if (loss) *loss = Lc.real();
  return Lc.imag() / h;
}

// Store-all reverse sweep of the same g-only run: full gradient of the loss
// with respect to tau[batch], the inflow state (e_in, beta_in[3]) and the
// initial fields e0[cells], beta0[3][cells].  Returns the loss.
double ora_gradient(const int32_t *dims, double c_l, const int32_t *bc, const double *inflow,
                    const uint8_t *solid, const OraRelax *rxp, const double *e0,
                    const double *beta0, int nsteps, const double *la, const double *lt,
                    const double *lbe, const double *lbb, double *g_tau, double *g_inflow,
                    double *g_e0, double *g_beta0, double *g_tau_cell) {
  const Relax<double> rx = relax_of(rxp);
  Lattice L = make_lattice(dims, c_l, bc);
  L.kappa = kappa_of(rxp->kappa);
  const long C = L.cells();
  const long QC = (long)Q * C;
  double in_f[Q], in_g[Q];
  inflow_equilibria<double>(L, inflow[0], inflow[1], inflow + 2, in_f, in_g);
  std::vector<double> states((long)(nsteps + 1) * QC);
  init_state<double>(L, solid, nullptr, e0, beta0, in_f, in_g, states.data(), false);
  for (int t = 0; t < nsteps; ++t)
    step<double>(L, rx, solid, in_f, in_g, states.data() + t * QC, states.data() + (t + 1) * QC,
                 false);
  const double *ST = states.data() + (long)nsteps * QC;
  std::vector<double> e(C), bt(3 * C);
  fields<double>(L, solid, ST, false, nullptr, e.data(), bt.data());
  LossSpec ls{la, lt, lbe, lbb};
  double Lv = loss_value<double>(L, solid, e.data(), bt.data(), ls);
  // dL/de and dL/dbeta of the loss, written out from its definition.
  std::vector<double> dLde(C, 0.0), dLdb(3 * C, 0.0);
  for (long i = 0; i < C; ++i) {
    if (solid && solid[i]) continue;
    if (la) dLde[i] += 2.0 * la[i] * (e[i] - lt[i]);
    if (lbe) dLde[i] += lbe[i];
    if (lbb)
      for (int k = 0; k < 3; ++k) dLdb[k * C + i] = lbb[k * C + i];
  }
  std::vector<double> lam(QC), lam2(QC);
  moments_adjoint_g(L, solid, ST, dLde.data(), dLdb.data(), lam.data());
  for (int b = 0; b < L.batch; ++b) g_tau[b] = 0.0;
  for (int k = 0; k < 4; ++k) g_inflow[k] = 0.0;
  if (g_tau_cell)
    for (long i = 0; i < C; ++i) g_tau_cell[i] = 0.0;
  for (int t = nsteps - 1; t >= 0; --t) {
    adjoint_step_g(L, rx, solid, inflow[1], inflow + 2, states.data() + t * QC, lam.data(),
                   lam2.data(), g_tau, g_inflow + 1, g_inflow, g_tau_cell);
    std::swap(lam, lam2);
  }
  init_adjoint_g(L, solid, e0, beta0, inflow[1], inflow + 2, lam.data(), g_e0, g_beta0,
                 g_inflow + 1, g_inflow);
  return Lv;
}

// Transport quantities of a stored f+g state per cell (zeros on solid
// cells): temperature, entropy density, shear viscosity and eta/s, with each
// cell's relaxation time from the relaxation source (for eta_s > 0 the tau
// that the rule gives at the cell's own fields).
int ora_transport(const int32_t *dims, double c_l, const uint8_t *solid, const double *S,
                  const OraRelax *rxp, double *temp, double *s, double *eta, double *eta_over_s) {
  const Relax<double> rx = relax_of(rxp);
  int32_t bc0[6] = {0, 0, 0, 0, 0, 0};
  Lattice L = make_lattice(dims, c_l, bc0);
  L.kappa = kappa_of(rxp->kappa);
  if (!radiation(L.kappa)) return 0;  // T = e/(3n) and n_eq are those of e = 3P matter
  const long C = L.cells();
  const long per = (long)L.n[0] * L.n[1] * L.n[2];
  for (long i = 0; i < C; ++i) {
    temp[i] = s[i] = eta[i] = eta_over_s[i] = 0.0;
    if (solid && solid[i]) continue;
    double pf[Q], pg[Q];
    for (int q = 0; q < Q; ++q) {
      pf[q] = S[(long)q * C + i];
      pg[q] = S[(long)(Q + q) * C + i];
    }
    double N, E, M[3], n, eps, beta[3];
    moment_sums(pf, pg, c_l, &N, &E, M);
    invert(N, E, M, &n, &eps, beta);
    double tau = rx.tau_cell ? rx.tau_cell[i] : rx.tau[i / per];
    if (rx.eta_s > 0.0) tau = tau_for_eta_s(pf, pg, c_l, rx.eta_s, rx.d_G);
    transport(n, eps, beta, tau, c_l, rx.d_G, &temp[i], &s[i], &eta[i]);
    eta_over_s[i] = eta[i] / s[i];
  }
  return 1;
}

}  // extern "C"

namespace {
Relax<double> relax_of(const void *r) {
  const OraRelax *x = static_cast<const OraRelax *>(r);
  return Relax<double>{x->tau, x->tau_cell, x->eta_s, x->d_G};
}
}  // namespace
