// Host side of librlb.so: parameter validation, launch geometry, storage
// dispatch and the C entry points declared in include/rlb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rlb.h"
#include "kernels.hpp"

// Loop entry points with at least this many steps replay a cached HIP graph
// of their launches (kernels only), from the second call with the same
// arguments on, instead of launching step by step.
constexpr int kGraphMin = 4;
constexpr int kGraphSlots = 12;
constexpr int kSeenSlots = 16;

using namespace rlb;

// Device-resident workspace of the allocation-free entry point
// (rlb_moments_noalloc): per-workgroup reduction partials, 5 doubles per
// workgroup.  Every device the library runs on holds its own copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (kept in
// g_scratch_addr), never through the array's name.
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};
}  // namespace

struct rlb_solver {
  rlb_params p;
  Geom g;
  Phys ph;
  InflowState in;
  Faces faces;
  int face_mode;  // FACES_* of the reverse gather
  int st, cp;
  size_t elem, lam_elem;
  void *pop[2];
  int cur;
  hipStream_t stream;
  double *d_omega;
  uint32_t *d_cls;
  void *d_in_eq;
  unsigned char in_eq_host[2 * Q * 8];  // the same values, read back once at init
  unsigned long long *d_counters;
  double *d_part;      // per-workgroup partials of moments / init-adjoint reductions
  double *d_part_rev;  // reverse-step partials of the streaming kernel (accumulated)
  double *d_inst;      // [batch][4] per-instance inflow partials
  double *d_res;
  void *d_scratch;   // one lambda block (reader form of single reverse steps)
  bool rev_pending;  // reverse-step partials accumulated and not yet reduced
  bool held;         // solid cells or an inflow plane exist (held cells)
  double *d_omega_cell;       // per-cell 1/tau of a tau field (or null)
  double *d_dtau_cell;        // per-cell dL/dtau(x) accumulated by the reverse steps
  unsigned long long *d_bad;  // validation counter of rlb_set_tau_field
  bool inplace;               // one state buffer, AA-pattern streaming
  int aa_phase;               // 0: swapped layout (S_t readable), 1: streamed layout
  void *d_fb;                 // face copies of the in-place layout
  FaceMap fm;
  int *d_aalist;              // cells of the in-place general path
  int n_aablk;
  int device;                 // device current at rlb_init
  double *d_static;           // that device's copy of `scratch` (its device address)
  // Loops of launches replayed as HIP graphs (one per distinct call signature)
  hipStream_t cap;            // private stream the loops are captured on
  struct GraphEntry {
    int kind;                 // 0 none, 1 advance, 2 trajectory, 3 reverse segment
    const void *a, *b, *c, *d;
    int64_t stride;
    int n, flags;
    hipGraphExec_t exec;
  } graphs[kGraphSlots], seen[kSeenSlots];  // seen: keys launched once, not captured
  int graph_next, seen_next;
};

namespace {

thread_local std::string g_err;

constexpr size_t kCounterBytes = sizeof(unsigned long long) * 2 * NSLOT * CSTRIDE;

rlb_status fail(rlb_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define RLB_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(RLB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

size_t elem_size(int st) {
  switch (st) {
    case ST_F64: return 8;
    case ST_F32:
    case ST_F32DEV: return 4;
    case ST_F16DEV:
    case ST_BF16DEV: return 2;
  }
  return 0;
}

FastDiv make_div(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}

long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

rlb_status validate(const rlb_params *p, long long *cells_out) {
  if (!p) return fail(RLB_EINVAL, "params is NULL");
  const int n[3] = {p->nx, p->ny, p->nz};
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->batch < 1)
    return fail(RLB_EINVAL, "extents and batch must be >= 1");
  const long long cells = (long long)p->nx * p->ny * p->nz * p->batch;
  if (cells > (1ll << 31) - 64) return fail(RLB_EINVAL, "too many cells (max 2^31 - 64)");
  if (!(p->c_l > 0.0) || !std::isfinite(p->c_l)) return fail(RLB_EINVAL, "c_l must be > 0");
  int inflow_faces = 0;
  for (int a = 0; a < 3; ++a) {
    for (int s = 0; s < 2; ++s) {
      int b = p->bc[a][s];
      if (b != RLB_BC_PERIODIC && b != RLB_BC_OUTFLOW && b != RLB_BC_INFLOW)
        return fail(RLB_EINVAL, "unknown boundary code");
      if (b == RLB_BC_INFLOW) ++inflow_faces;
    }
    if ((p->bc[a][0] == RLB_BC_PERIODIC) != (p->bc[a][1] == RLB_BC_PERIODIC))
      return fail(RLB_EINVAL, "an axis is periodic on both faces or on neither");
    if (p->bc[a][0] != RLB_BC_PERIODIC && n[a] < 2)
      return fail(RLB_EINVAL, "a non-periodic axis needs at least 2 cells");
  }
  if (inflow_faces > 1) return fail(RLB_EINVAL, "at most one INFLOW face");
  if (inflow_faces == 1) {
    double b2 = p->inflow_beta[0] * p->inflow_beta[0] + p->inflow_beta[1] * p->inflow_beta[1] +
                p->inflow_beta[2] * p->inflow_beta[2];
    if (!(p->inflow_e > 0.0) || !std::isfinite(p->inflow_e))
      return fail(RLB_EINVAL, "inflow_e must be > 0");
    if (!(b2 < 1.0)) return fail(RLB_EINVAL, "|inflow_beta| must be < 1");
    if (!std::isfinite(p->inflow_n)) return fail(RLB_EINVAL, "inflow_n must be finite");
  }
  if (elem_size(p->storage) == 0) return fail(RLB_EINVAL, "unknown storage");
  if (p->collide != RLB_COLLIDE_AUTO && p->collide != RLB_COLLIDE_F32 &&
      p->collide != RLB_COLLIDE_F64 && p->collide != RLB_COLLIDE_F32_MOM64)
    return fail(RLB_EINVAL, "unknown collision type");
  if (p->storage == RLB_F64 && (p->collide == RLB_COLLIDE_F32 || p->collide == RLB_COLLIDE_F32_MOM64))
    return fail(RLB_EINVAL, "FP64 storage collides in FP64");
  if ((p->storage == RLB_F16DEV || p->storage == RLB_BF16DEV) && p->collide == RLB_COLLIDE_F32_MOM64)
    return fail(RLB_EINVAL, "FP64 moment sums are offered with the 4-byte storages");
  if ((p->storage == RLB_F16DEV || p->storage == RLB_BF16DEV) && p->collide == RLB_COLLIDE_F64)
    return fail(RLB_EINVAL, "16-bit storages collide in FP32");
  if (p->storage >= ST_F32DEV) {
    if (!(p->e_ref > 0.0) || !std::isfinite(p->e_ref) || !std::isfinite(p->n_ref))
      return fail(RLB_EINVAL, "deviation storage needs e_ref > 0 and finite n_ref");
  }
  if (!(p->kappa == 0.0 || (p->kappa > 0.0 && p->kappa <= 1.0)))
    return fail(RLB_EINVAL, "kappa (P = kappa e) must be in (0, 1], or 0 for 1/3");
  if (p->inplace != 0 && p->inplace != 1) return fail(RLB_EINVAL, "inplace must be 0 or 1");
  *cells_out = cells;
  return RLB_OK;
}

void setup_geometry(rlb_solver *h) {
  const rlb_params &p = h->p;
  Geom &g = h->g;
  std::memset(&g, 0, sizeof(g));
  g.n[0] = p.nx;
  g.n[1] = p.ny;
  g.n[2] = p.nz;
  g.batch = p.batch;
  g.per = p.nx * p.ny * p.nz;
  g.nblk_per = (g.per + BLOCK - 1) / BLOCK;
  g.nblk = g.nblk_per * p.batch;
  g.qs = round_up((long long)g.per * p.batch, 64);
  g.div_x = make_div((uint32_t)p.nx);
  g.div_y = make_div((uint32_t)p.ny);
  g.div_blk = make_div((uint32_t)g.nblk_per);
  const int stride[3] = {1, p.nx, p.nx * p.ny};
  for (int a = 0; a < 3; ++a) {
    g.periodic[a] = p.bc[a][0] == RLB_BC_PERIODIC;
    g.inflow_lo[a] = p.bc[a][0] == RLB_BC_INFLOW;
    g.inflow_hi[a] = p.bc[a][1] == RLB_BC_INFLOW;
    if (g.inflow_lo[a] || g.inflow_hi[a]) g.any_inflow = 1;
    if (g.periodic[a]) {
      // wrap; on an axis of one cell every pull returns to the cell itself
      g.corr_lo[a] = g.n[a] == 1 ? 0 : g.n[a] * stride[a];
      g.corr_hi[a] = g.n[a] == 1 ? 0 : -g.n[a] * stride[a];
    } else {
      // clamp onto the face (zero-gradient copy)
      g.corr_lo[a] = stride[a];
      g.corr_hi[a] = -stride[a];
    }
  }
  const int e[Q][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                       {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                       {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                       {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  for (int q = 0; q < Q; ++q) {
    int o = 0;
    for (int a = 0; a < 3; ++a)
      if (!(g.periodic[a] && g.n[a] == 1)) o += e[q][a] * stride[a];
    g.off[q] = o;
  }
  Faces &F = h->faces;
  std::memset(&F, 0, sizeof(F));
  long long acc = 0;
  for (int a = 0; a < 3; ++a) {
    if (g.periodic[a]) continue;
    const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
    for (int s = 0; s < 2; ++s) {
      F.axis[F.count] = a;
      F.side[F.count] = s;
      F.start[F.count] = acc;
      acc += (long long)p.batch * g.n[u] * g.n[v];
      ++F.count;
    }
  }
  F.start[F.count] = acc;
  // one non-periodic axis of extent > 1: the reverse gather specialised to it
  int np_axes = 0, np_axis = -1;
  for (int a = 0; a < 3; ++a)
    if (!g.periodic[a]) {
      ++np_axes;
      np_axis = a;
    }
  h->face_mode = np_axes == 0 ? FACES_NONE
                 : (np_axes == 1 && g.n[np_axis] > 1) ? FACES_X + np_axis
                                                      : FACES_ANY;
}

unsigned grid_blocks(const rlb_solver *h) { return (unsigned)h->g.nblk; }

template <int ST, class TC>
rlb_status launch_init(rlb_solver *h, const double *n0, const double *e0, const double *beta0) {
  using El = typename Codec<ST, TC>::elem;
  const rlb_params &p = h->p;
  hipLaunchKernelGGL((k_inflow_eq<ST, TC>), dim3(1), dim3(64), 0, h->stream, h->ph, p.inflow_n,
                     p.inflow_e, p.inflow_beta[0], p.inflow_beta[1], p.inflow_beta[2],
                     (El *)h->d_in_eq);
  hipLaunchKernelGGL((k_init<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g, h->ph,
                     n0, e0, beta0, (El *)h->pop[0], (El *)h->pop[1], (const El *)h->d_in_eq);
  if (h->inplace)
    hipLaunchKernelGGL((k_aa_swap<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g,
                       h->ph, h->fm, (El *)h->pop[0], (El *)h->d_fb);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

template <class El>
HeldEq<El> held_eq(const rlb_solver *h) {
  HeldEq<El> v;
  static_assert(sizeof(v.v) <= sizeof(h->in_eq_host), "held values exceed the host copy");
  std::memcpy(v.v, h->in_eq_host, sizeof(v.v));
  return v;
}

// Two cells per lane (k_step_pairs): FP64 storage, or FP32 / FP32-deviation
// storage with FP64 collision; an even x extent, no held cells, no eta/s
// rule.  Returns whether it launched.
template <int ST, class TC>
bool launch_step_pairs(rlb_solver *h, const typename Codec<ST, TC>::elem *src,
                       typename Codec<ST, TC>::elem *dst) {
  constexpr bool pairs = ST == ST_F64 ||
                         ((ST == ST_F32 || ST == ST_F32DEV) && std::is_same<TC, double>::value);
  if constexpr (!pairs) {
    return false;
  } else {
    if (h->held || h->ph.eta_s > 0.0 || h->g.n[0] % 2 != 0) return false;
    const int npb = (h->g.per / 2 + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL((k_step_pairs<ST, TC>), dim3(npb * h->g.batch), dim3(BLOCK), 0, h->stream,
                       h->g, h->ph, npb, src, dst, h->d_counters);
    return true;
  }
}

template <int ST, class TC>
rlb_status launch_steps(rlb_solver *h, int nsteps) {
  using El = typename Codec<ST, TC>::elem;
  const HeldEq<El> in_eq = held_eq<El>(h);
  if (h->inplace) {
    El *A = (El *)h->pop[0];
    for (int s = 0; s < nsteps; ++s) {
      if (h->aa_phase == 0) {
        // listed cells (general path) and the rest (fast path) in one launch
        hipLaunchKernelGGL((k_aa_pull_all<ST, TC>), dim3(h->n_aablk + grid_blocks(h)), dim3(BLOCK),
                           0, h->stream, h->g, h->ph, h->fm, h->n_aablk,
                           (const int *)h->d_aalist, A, (const El *)h->d_fb, in_eq,
                           h->d_counters);
      } else
        hipLaunchKernelGGL((k_aa_local<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream,
                           h->g, h->ph, h->fm, A, (El *)h->d_fb, in_eq, h->d_counters);
      h->aa_phase = 1 - h->aa_phase;
    }
    RLB_HIP(hipGetLastError());
    return RLB_OK;
  }
  for (int s = 0; s < nsteps; ++s) {
    const El *src = (const El *)h->pop[h->cur];
    El *dst = (El *)h->pop[1 - h->cur];
    const bool etas = h->ph.eta_s > 0.0;
    if (h->held && etas)
      hipLaunchKernelGGL((k_step<ST, TC, true, true, true>), dim3(grid_blocks(h)), dim3(BLOCK), 0,
                         h->stream, h->g, h->ph, src, dst, in_eq, h->d_counters);
    else if (h->held)
      hipLaunchKernelGGL((k_step<ST, TC, true, true>), dim3(grid_blocks(h)), dim3(BLOCK), 0,
                         h->stream, h->g, h->ph, src, dst, in_eq, h->d_counters);
    else if (etas)
      hipLaunchKernelGGL((k_step<ST, TC, true, false, true>), dim3(grid_blocks(h)), dim3(BLOCK),
                         0, h->stream, h->g, h->ph, src, dst, in_eq, h->d_counters);
    else if (launch_step_pairs<ST, TC>(h, src, dst)) {
    } else
      hipLaunchKernelGGL((k_step<ST, TC, true, false>), dim3(grid_blocks(h)), dim3(BLOCK), 0,
                         h->stream, h->g, h->ph, src, dst, in_eq, h->d_counters);
    h->cur = 1 - h->cur;
  }
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

template <int ST, class TC>
rlb_status launch_step_g(rlb_solver *h, const void *src, void *dst) {
  using El = typename Codec<ST, TC>::elem;
  if (h->held)
    hipLaunchKernelGGL((k_step<ST, TC, false, true>), dim3(grid_blocks(h)), dim3(BLOCK), 0,
                       h->stream, h->g, h->ph, (const El *)src, (El *)dst, held_eq<El>(h),
                       h->d_counters);
  else
    hipLaunchKernelGGL((k_step<ST, TC, false, false>), dim3(grid_blocks(h)), dim3(BLOCK), 0,
                       h->stream, h->g, h->ph, (const El *)src, (El *)dst, held_eq<El>(h),
                       h->d_counters);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

template <int ST, class TC>
rlb_status launch_transport(rlb_solver *h, double *T, double *ent, double *eta, double *eos) {
  using El = typename Codec<ST, TC>::elem;
  const El *S = (const El *)h->pop[h->cur];
  hipLaunchKernelGGL((k_transport<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g,
                     h->ph, S, S + (size_t)Q * h->g.qs, T, ent, eta, eos, h->inplace ? 1 : 0);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

// Fields of the current state and, with part != null, its conservation sums
// reduced through the per-workgroup partials `part` (5 per workgroup) into
// res[batch][5] (device).
template <int ST, class TC>
rlb_status launch_moments(rlb_solver *h, double *n, double *e, double *beta, double *part,
                          double *res) {
  using El = typename Codec<ST, TC>::elem;
  const El *S = (const El *)h->pop[h->cur];
  hipLaunchKernelGGL((k_moments<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g, h->ph,
                     S, S + (size_t)Q * h->g.qs, n, e, beta, part, h->inplace ? 1 : 0);
  if (part)
    hipLaunchKernelGGL(k_finish, dim3(h->p.batch), dim3(BLOCK), 0, h->stream, part,
                       h->g.nblk_per, (const double *)nullptr, (const int *)nullptr, res,
                       (double *)nullptr, (double *)nullptr);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

template <int ST, class TC>
rlb_status launch_fields_g(rlb_solver *h, const void *Sg, double *e, double *beta) {
  using El = typename Codec<ST, TC>::elem;
  hipLaunchKernelGGL((k_moments<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g, h->ph,
                     (const El *)nullptr, (const El *)Sg, (double *)nullptr, e, beta,
                     (double *)nullptr, 0);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

// Cells of the general reverse path, in index order, each instance padded to
// whole workgroups (-1 entries), so that every workgroup's partial sums belong
// to one instance and their reduction order is fixed.
// Cells of the in-place general path (flagged by k_mark_aa), in index order,
// padded to whole workgroups.
rlb_status build_aa_list(rlb_solver *h) {
  const size_t cells = (size_t)h->g.per * h->p.batch;
  uint8_t *d_flag = nullptr;
  RLB_HIP(hipMalloc(&d_flag, cells));
  hipLaunchKernelGGL(k_mark_aa, dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g, h->ph,
                     d_flag);
  std::vector<uint8_t> flag(cells);
  hipError_t e = hipMemcpyAsync(flag.data(), d_flag, cells, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(d_flag);
  if (e != hipSuccess) return fail(RLB_EDEVICE, std::string("in-place list: ") + hipGetErrorString(e));
  std::vector<int> list;
  for (size_t i = 0; i < cells; ++i)
    if (flag[i]) list.push_back((int)i);
  if (!list.empty())
    while (list.size() % (8 * BLOCK)) list.push_back(-1);  // whole XCD rounds of workgroups
  h->n_aablk = (int)(list.size() / BLOCK);
  if (h->n_aablk > 0) {
    RLB_HIP(hipMalloc(&h->d_aalist, list.size() * sizeof(int)));
    RLB_HIP(hipMemcpy(h->d_aalist, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  return RLB_OK;
}

void drop_graphs(rlb_solver *h) {
  for (int i = 0; i < kGraphSlots; ++i)
    if (h->graphs[i].kind) {
      (void)hipGraphExecDestroy(h->graphs[i].exec);
      h->graphs[i].kind = 0;
    }
}

// Run `body` (which launches on h->stream) through a cached graph keyed by
// (kind, a, b, c, stride, n): launched directly the first time a key is seen,
// captured on a private stream the second time, replayed on h->stream
// afterwards (calls whose buffers never repeat pay no capture).  Kernel
// arguments (geometry, physics, buffers) are fixed at capture; anything that
// changes them drops the cache.
template <class F>
rlb_status run_graph(rlb_solver *h, int kind, const void *a, const void *b, const void *c,
                     const void *d, int64_t stride, int n, int flags, F body) {
  auto same = [&](const rlb_solver::GraphEntry &G) {
    return G.kind == kind && G.a == a && G.b == b && G.c == c && G.d == d &&
           G.stride == stride && G.n == n && G.flags == flags;
  };
  for (int i = 0; i < kGraphSlots; ++i) {
    const auto &G = h->graphs[i];
    if (same(G)) {
      RLB_HIP(hipGraphLaunch(G.exec, h->stream));
      return RLB_OK;
    }
  }
  bool seen = false;
  for (int i = 0; i < kSeenSlots && !seen; ++i) {
    auto &K = h->seen[i];
    if (same(K)) {
      seen = true;
      K.kind = 0;
    }
  }
  if (!seen) {
    h->seen[h->seen_next] = {kind, a, b, c, d, stride, n, flags, nullptr};
    h->seen_next = (h->seen_next + 1) % kSeenSlots;
    return body();
  }
  if (!h->cap) RLB_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  hipStream_t user = h->stream;
  RLB_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  h->stream = h->cap;
  rlb_status st = body();
  h->stream = user;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap, &graph);
  if (st != RLB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(RLB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess)
    return fail(RLB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  auto &G = h->graphs[h->graph_next];
  if (G.kind) (void)hipGraphExecDestroy(G.exec);
  G = {kind, a, b, c, d, stride, n, flags, exec};
  h->graph_next = (h->graph_next + 1) % kGraphSlots;
  RLB_HIP(hipGraphLaunch(exec, h->stream));
  return RLB_OK;
}

// One reverse step into the reader form R_out (see k_adjoint): lambda_{t+1}
// from lam_in, natural (nat_in) or in reader form.  Its partial sums are added
// to the pending ones.
template <int ST, class TC>
rlb_status launch_adjoint(rlb_solver *h, const void *S, const void *lam_in, bool nat_in,
                          void *R_out) {
  using El = typename Codec<ST, TC>::elem;
  const int accum = h->rev_pending ? 1 : 0;
  const dim3 grid(grid_blocks(h)), block(BLOCK);
  const El *s = (const El *)S;
  const LamT *li = (const LamT *)lam_in;
  LamT *ro = (LamT *)R_out;
#define RLB_ADJ(NAT, FM)                                                                       \
  hipLaunchKernelGGL((k_adjoint<ST, TC, NAT, FM>), grid, block, 0, h->stream, h->g, h->ph, s, li, \
                     ro, h->d_part_rev, h->in, accum)
  if (nat_in) {
    RLB_ADJ(true, FACES_NONE);  // a natural input reads no neighbours
  } else {
    switch (h->face_mode) {
      case FACES_NONE: RLB_ADJ(false, FACES_NONE); break;
      case FACES_X: RLB_ADJ(false, FACES_X); break;
      case FACES_Y: RLB_ADJ(false, FACES_Y); break;
      case FACES_Z: RLB_ADJ(false, FACES_Z); break;
      default: RLB_ADJ(false, FACES_ANY); break;
    }
  }
#undef RLB_ADJ
  h->rev_pending = true;
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

// Natural lambda from its reader form.
rlb_status launch_lam_gather(rlb_solver *h, const void *R, void *lam) {
  const dim3 grid(grid_blocks(h)), block(BLOCK);
  const LamT *r = (const LamT *)R;
  LamT *l = (LamT *)lam;
  switch (h->face_mode) {
    case FACES_NONE:
      hipLaunchKernelGGL(k_lam_gather<FACES_NONE>, grid, block, 0, h->stream, h->g, h->ph, r, l);
      break;
    case FACES_X:
      hipLaunchKernelGGL(k_lam_gather<FACES_X>, grid, block, 0, h->stream, h->g, h->ph, r, l);
      break;
    case FACES_Y:
      hipLaunchKernelGGL(k_lam_gather<FACES_Y>, grid, block, 0, h->stream, h->g, h->ph, r, l);
      break;
    case FACES_Z:
      hipLaunchKernelGGL(k_lam_gather<FACES_Z>, grid, block, 0, h->stream, h->g, h->ph, r, l);
      break;
    default:
      hipLaunchKernelGGL(k_lam_gather<FACES_ANY>, grid, block, 0, h->stream, h->g, h->ph, r, l);
      break;
  }
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

// Reduce the pending reverse-step partials (fixed order) into the gradients.
rlb_status flush_adjoint(rlb_solver *h, double *dtau, double *dbeta_in, double *de_in) {
  if (!h->rev_pending) return RLB_OK;
  hipLaunchKernelGGL(k_finish, dim3(h->p.batch), dim3(BLOCK), 0, h->stream, h->d_part_rev,
                     h->g.nblk_per, (const double *)nullptr, (const int *)nullptr,
                     (double *)nullptr, dtau, h->d_inst);
  if (dbeta_in || de_in)
    hipLaunchKernelGGL(k_finish_inflow, dim3(1), dim3(64), 0, h->stream, (const double *)h->d_inst,
                       h->p.batch, de_in, dbeta_in);
  h->rev_pending = false;
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

// Start the pending reverse-step partials at zero (a kernel, not a memset, so
// that it may sit in a captured graph), so that steps may always accumulate.
rlb_status zero_reverse_partials(rlb_solver *h) {
  const long long n1 = 5LL * h->g.nblk;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n1 + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, h->stream,
                     h->d_part_rev, n1);
  h->rev_pending = true;
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

template <int ST, class TC>
rlb_status launch_moments_adjoint(rlb_solver *h, const void *S, const double *dLde,
                                  const double *dLdb, void *lam) {
  using El = typename Codec<ST, TC>::elem;
  using Lm = typename Codec<ST, TC>::lam;
  hipLaunchKernelGGL((k_moments_adjoint<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream,
                     h->g, h->ph, (const El *)S, dLde, dLdb, (Lm *)lam);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

template <int ST, class TC>
rlb_status launch_init_adjoint(rlb_solver *h, const double *e0, const double *beta0,
                               const void *lam0, double *de0, double *db0, double *dbeta_in,
                               double *de_in) {
  using Lm = typename Codec<ST, TC>::lam;
  hipLaunchKernelGGL((k_init_adjoint<ST, TC>), dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g,
                     h->ph, e0, beta0, (const Lm *)lam0, de0, db0, h->d_part, h->in);
  if (dbeta_in || de_in) {
    hipLaunchKernelGGL(k_finish, dim3(h->p.batch), dim3(BLOCK), 0, h->stream, h->d_part,
                       h->g.nblk_per, (const double *)nullptr, (const int *)nullptr,
                       (double *)nullptr, (double *)nullptr, h->d_inst);
    hipLaunchKernelGGL(k_finish_inflow, dim3(1), dim3(64), 0, h->stream, (const double *)h->d_inst,
                       h->p.batch, de_in, dbeta_in);
  }
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

// Storage x compute-type dispatch: RLB_DISPATCH(h, fn, args...) calls
// fn<ST, TC>(args...) for the solver's storage and collision type.
#define RLB_DISPATCH(h, fn, ...)                                                   \
  do {                                                                             \
    const bool c64_ = (h)->cp == RLB_COLLIDE_F64;                                  \
    const bool s64_ = (h)->cp == RLB_COLLIDE_F32_MOM64;                            \
    switch ((h)->st) {                                                             \
      case ST_F64: return fn<ST_F64, double>(__VA_ARGS__);                         \
      case ST_F32:                                                                 \
        return c64_ ? fn<ST_F32, double>(__VA_ARGS__)                              \
                    : (s64_ ? fn<ST_F32, f32s>(__VA_ARGS__) : fn<ST_F32, float>(__VA_ARGS__)); \
      case ST_F32DEV:                                                              \
        return c64_ ? fn<ST_F32DEV, double>(__VA_ARGS__)                           \
                    : (s64_ ? fn<ST_F32DEV, f32s>(__VA_ARGS__)                     \
                            : fn<ST_F32DEV, float>(__VA_ARGS__));                  \
      case ST_F16DEV: return fn<ST_F16DEV, float>(__VA_ARGS__);                    \
      case ST_BF16DEV: return fn<ST_BF16DEV, float>(__VA_ARGS__);                  \
    }                                                                              \
    return fail(RLB_EINVAL, "unknown storage");                                    \
  } while (0)

// Resolved collision type: AUTO is FP64 for the 8- and 4-byte storages (the
// FP32 rounding of the collision itself would dominate their error) and FP32
// for the 2-byte storages (their storage rounding dominates).
int resolve_collide(const rlb_params *p) {
  if (p->collide != RLB_COLLIDE_AUTO) return p->collide;
  return (p->storage == RLB_F16DEV || p->storage == RLB_BF16DEV) ? RLB_COLLIDE_F32
                                                                 : RLB_COLLIDE_F64;
}

void free_solver(rlb_solver *h) {
  if (!h) return;
  if (h->d_omega) (void)hipFree(h->d_omega);
  if (h->d_cls) (void)hipFree(h->d_cls);
  if (h->d_in_eq) (void)hipFree(h->d_in_eq);
  if (h->d_counters) (void)hipFree(h->d_counters);
  if (h->d_part) (void)hipFree(h->d_part);
  if (h->d_part_rev) (void)hipFree(h->d_part_rev);
  if (h->d_inst) (void)hipFree(h->d_inst);
  if (h->d_res) (void)hipFree(h->d_res);
  if (h->d_scratch) (void)hipFree(h->d_scratch);
  if (h->d_omega_cell) (void)hipFree(h->d_omega_cell);
  if (h->d_dtau_cell) (void)hipFree(h->d_dtau_cell);
  if (h->d_bad) (void)hipFree(h->d_bad);
  if (h->d_fb) (void)hipFree(h->d_fb);
  if (h->d_aalist) (void)hipFree(h->d_aalist);
  for (int i = 0; i < kGraphSlots; ++i)
    if (h->graphs[i].kind) (void)hipGraphExecDestroy(h->graphs[i].exec);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  delete h;
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept for later calls.
rlb_status static_scratch(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(RLB_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(RLB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e));
    g_scratch_addr[dev] = (double *)ptr;
  }
  *out = g_scratch_addr[dev];
  return RLB_OK;
}

rlb_status check_handle(const rlb_solver *h) {
  if (!h) return fail(RLB_EINVAL, "solver handle is NULL");
  return RLB_OK;
}

}  // namespace

extern "C" {

rlb_status rlb_buffer_layout(const rlb_params *p, int64_t *q_stride, int64_t *state_bytes) {
  long long cells = 0;
  rlb_status s = validate(p, &cells);
  if (s != RLB_OK) return s;
  const long long qs = round_up(cells, 64);
  if (q_stride) *q_stride = qs;
  if (state_bytes) *state_bytes = 2LL * Q * qs * (long long)elem_size(p->storage);
  return RLB_OK;
}

rlb_status rlb_init(rlb_solver **out, const rlb_params *p, const double *tau,
                    const uint8_t *solid, const double *n0, const double *e0,
                    const double *beta0, void *pop_a, void *pop_b, void *stream) {
  g_err.clear();
  if (!out) return fail(RLB_EINVAL, "out is NULL");
  *out = nullptr;
  long long cells = 0;
  rlb_status s = validate(p, &cells);
  if (s != RLB_OK) return s;
  const bool inplace = p->inplace != 0;
  if (!tau || !n0 || !e0 || !beta0 || !pop_a || (!inplace && !pop_b))
    return fail(RLB_EINVAL, "a required pointer is NULL");
  if (!inplace && pop_a == pop_b) return fail(RLB_EINVAL, "pop_a and pop_b must differ");
  for (int b = 0; b < p->batch; ++b)
    if (!(tau[b] > 0.5) || !std::isfinite(tau[b]))
      return fail(RLB_EINVAL, "tau must be > 1/2 (positive viscosity) for every instance");

  rlb_solver *h = new rlb_solver;
  std::memset(h, 0, sizeof(*h));
  h->p = *p;
  h->st = p->storage;
  h->cp = resolve_collide(p);
  h->elem = elem_size(p->storage);
  h->lam_elem = sizeof(LamT);
  h->pop[0] = pop_a;
  h->pop[1] = inplace ? pop_a : pop_b;  // the in-place layout uses pop_a only
  h->inplace = inplace;
  h->aa_phase = 0;
  h->cur = 0;
  h->stream = (hipStream_t)stream;
  setup_geometry(h);

  Phys &ph = h->ph;
  ph.c = p->c_l;
  ph.inv_c = 1.0 / p->c_l;
  ph.inv_c2 = 1.0 / (p->c_l * p->c_l);
  ph.k0 = 3.0 - 2.0 / (p->c_l * p->c_l);
  ph.ad_c = ph.inv_c2;
  ph.wfac = 4.0 / 3.0;
  ph.kappa = 1.0 / 3.0;
  ph.gen_eos = 0;
  ph.eos_A = 4.0;
  ph.eos_B = 3.0;
  ph.eos_C = 2.0;
  ph.eos_H = 1.0 / 3.0;
  ph.eos_F = 1.0;
  ph.eos_G = 1.0;
  if (p->kappa != 0.0 && p->kappa != 1.0 / 3.0) {
    // P = kappa e: eqs. (equil2a)/(equil2b) in the same W-form
    const double k = p->kappa;
    ph.kappa = k;
    ph.gen_eos = 1;
    ph.ad_c = 3.0 * k / (p->c_l * p->c_l);
    ph.k0 = 3.0 - 6.0 * k / (p->c_l * p->c_l);
    ph.wfac = 1.0 + k;
    ph.eos_A = (1.0 + k) * (1.0 + k);
    ph.eos_B = 4.0 * k;
    ph.eos_C = 1.0 + k;
    ph.eos_H = 0.5;
    ph.eos_F = 1.0 - k;
    ph.eos_G = 1.0 / (2.0 * k);
  }
  const bool dev = p->storage >= ST_F32DEV;
  ph.n_ref = dev ? p->n_ref : 0.0;
  ph.e_ref = dev ? p->e_ref : 0.0;
  ph.d_G = 16.0;
  h->in.e = p->inflow_e;
  h->in.bx = p->inflow_beta[0];
  h->in.by = p->inflow_beta[1];
  h->in.bz = p->inflow_beta[2];

  auto cleanup_fail = [&](hipError_t e, const char *what) {
    free_solver(h);
    return fail(RLB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&h->device)) != hipSuccess) return cleanup_fail(e, "hipGetDevice");
  if ((s = static_scratch(h->device, &h->d_static)) != RLB_OK) {
    free_solver(h);
    return s;
  }
  std::vector<double> om(p->batch);
  for (int b = 0; b < p->batch; ++b) om[b] = 1.0 / tau[b];
  if ((e = hipMalloc(&h->d_omega, sizeof(double) * p->batch)) != hipSuccess)
    return cleanup_fail(e, "hipMalloc(omega)");
  if ((e = hipMemcpyAsync(h->d_omega, om.data(), sizeof(double) * p->batch,
                          hipMemcpyHostToDevice, h->stream)) != hipSuccess)
    return cleanup_fail(e, "copy omega");
  if ((e = hipMalloc(&h->d_in_eq, 2 * Q * 8)) != hipSuccess)
    return cleanup_fail(e, "hipMalloc(inflow)");
  if ((e = hipMalloc(&h->d_counters, kCounterBytes)) != hipSuccess)
    return cleanup_fail(e, "hipMalloc(counters)");
  if ((e = hipMemsetAsync(h->d_counters, 0, kCounterBytes, h->stream)) != hipSuccess)
    return cleanup_fail(e, "clear counters");
  if ((e = hipMalloc(&h->d_part, sizeof(double) * 5 * (size_t)h->g.nblk)) != hipSuccess)
    return cleanup_fail(e, "hipMalloc(partials)");
  if ((e = hipMalloc(&h->d_part_rev, sizeof(double) * 5 * (size_t)h->g.nblk)) != hipSuccess)
    return cleanup_fail(e, "hipMalloc(reverse partials)");
  if ((e = hipMalloc(&h->d_inst, sizeof(double) * 4 * (size_t)p->batch)) != hipSuccess)
    return cleanup_fail(e, "hipMalloc(instance partials)");
  if ((e = hipMalloc(&h->d_res, sizeof(double) * 5 * (size_t)p->batch)) != hipSuccess)
    return cleanup_fail(e, "hipMalloc(results)");
  if (solid) {
    if ((e = hipMalloc(&h->d_cls, (size_t)h->g.qs * sizeof(uint32_t))) != hipSuccess)
      return cleanup_fail(e, "hipMalloc(classes)");
    hipLaunchKernelGGL(k_classify, dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g, solid,
                       h->d_cls);
    ph.cls = h->d_cls;
  }
  ph.omega = h->d_omega;
  h->held = solid != nullptr || h->g.any_inflow != 0;
  if (inplace) {
    FaceMap &fm = h->fm;
    for (int a = 0; a < 3; ++a) fm.id[a][0] = fm.id[a][1] = -1;
    for (int f = 0; f < h->faces.count; ++f) fm.id[h->faces.axis[f]][h->faces.side[f]] = f;
    for (int f = 0; f <= h->faces.count; ++f) fm.start[f] = h->faces.start[f];
    fm.count = h->faces.count;
    fm.nf = h->faces.start[h->faces.count];
    if (fm.nf > 0 &&
        (e = hipMalloc(&h->d_fb, (size_t)2 * Q * fm.nf * h->elem)) != hipSuccess)
      return cleanup_fail(e, "hipMalloc(face copies)");
    if ((s = build_aa_list(h)) != RLB_OK) {
      free_solver(h);
      return s;
    }
  }
  auto launch = [&]() -> rlb_status { RLB_DISPATCH(h, launch_init, h, n0, e0, beta0); };
  s = launch();
  if (s == RLB_OK && (e = hipStreamSynchronize(h->stream)) != hipSuccess)
    s = fail(RLB_EDEVICE, std::string("rlb_init: ") + hipGetErrorString(e));
  if (s == RLB_OK && (e = hipMemcpy(h->in_eq_host, h->d_in_eq, 2 * Q * h->elem,
                                    hipMemcpyDeviceToHost)) != hipSuccess)
    s = fail(RLB_EDEVICE, std::string("rlb_init: read inflow state: ") + hipGetErrorString(e));
  if (s != RLB_OK) {
    free_solver(h);
    return s;
  }
  *out = h;
  return RLB_OK;
}

rlb_status rlb_step(rlb_solver *h, int32_t nsteps) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (nsteps < 0) return fail(RLB_EINVAL, "nsteps must be >= 0");
  RLB_DISPATCH(h, launch_steps, h, nsteps);
}

rlb_status rlb_step_g(rlb_solver *h, const void *g_src, void *g_dst) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace) return fail(RLB_EINVAL, "the g-only and reverse entry points need the two-buffer layout (inplace = 0)");
  if (h->ph.eta_s > 0.0)
    return fail(RLB_EINVAL, "g-only steps and reverse steps are unavailable while eta/s is held");
  if (!g_src || !g_dst || g_src == g_dst) return fail(RLB_EINVAL, "g_src/g_dst invalid");
  RLB_DISPATCH(h, launch_step_g, h, g_src, g_dst);
}

rlb_status rlb_current(rlb_solver *h, void **state) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (!state) return fail(RLB_EINVAL, "state is NULL");
  *state = h->pop[h->cur];
  return RLB_OK;
}

rlb_status rlb_moments(rlb_solver *h, double *n, double *e, double *beta, double *sums) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace && h->aa_phase != 0)
    return fail(RLB_EINVAL, "in-place layout after an odd number of steps: S_t is not stored");
  double *part = sums ? h->d_part : nullptr;
  auto launch = [&]() -> rlb_status {
    RLB_DISPATCH(h, launch_moments, h, n, e, beta, part, h->d_res);
  };
  rlb_status s = launch();
  if (s != RLB_OK || !sums) return s;
  RLB_HIP(hipMemcpyAsync(sums, h->d_res, sizeof(double) * 5 * h->p.batch, hipMemcpyDeviceToHost,
                         h->stream));
  RLB_HIP(hipStreamSynchronize(h->stream));
  return RLB_OK;
}

rlb_status rlb_moments_noalloc(rlb_solver *h, double *n, double *e, double *beta,
                               double *sums) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace && h->aa_phase != 0)
    return fail(RLB_EINVAL, "in-place layout after an odd number of steps: S_t is not stored");
  if (!n && !e && !beta && !sums) return fail(RLB_EINVAL, "no output requested");
  const size_t need = (size_t)h->g.nblk * 5 * sizeof(double);
  if (sums && need > kStaticScratchBytes)
    return fail(RLB_EINVAL, "lattice too large for the static workspace: " +
                                std::to_string(h->g.nblk) + " workgroups need " +
                                std::to_string(need) + " bytes, the maximum is " +
                                std::to_string(kStaticScratchBytes));
  double *part = sums ? h->d_static : nullptr;
  RLB_DISPATCH(h, launch_moments, h, n, e, beta, part, sums);
}

rlb_status rlb_fields_g(rlb_solver *h, const void *g_state, double *e, double *beta) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace) return fail(RLB_EINVAL, "the g-only and reverse entry points need the two-buffer layout (inplace = 0)");
  if (!g_state || (!e && !beta)) return fail(RLB_EINVAL, "g_state or outputs invalid");
  RLB_DISPATCH(h, launch_fields_g, h, g_state, e, beta);
}

rlb_status rlb_counters(rlb_solver *h, int64_t counts[2]) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (!counts) return fail(RLB_EINVAL, "counts is NULL");
  std::vector<unsigned long long> buf(kCounterBytes / sizeof(unsigned long long));
  RLB_HIP(hipMemcpyAsync(buf.data(), h->d_counters, kCounterBytes, hipMemcpyDeviceToHost,
                         h->stream));
  RLB_HIP(hipStreamSynchronize(h->stream));
  RLB_HIP(hipMemsetAsync(h->d_counters, 0, kCounterBytes, h->stream));
  unsigned long long c[2] = {0, 0};
  for (int k = 0; k < 2; ++k)
    for (int i = 0; i < NSLOT; ++i) c[k] += buf[(size_t)(k * NSLOT + i) * CSTRIDE];
  counts[0] = (int64_t)c[0];
  counts[1] = (int64_t)c[1];
  return c[0] > 0 ? RLB_EUNPHYSICAL : RLB_OK;
}

static rlb_status check_reverse(rlb_solver *h) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace) return fail(RLB_EINVAL, "the g-only and reverse entry points need the two-buffer layout (inplace = 0)");
  if (h->ph.eta_s > 0.0)
    return fail(RLB_EINVAL, "g-only steps and reverse steps are unavailable while eta/s is held");
  return RLB_OK;
}

rlb_status rlb_adjoint_step(rlb_solver *h, const void *g_state_t, const void *lam_next,
                            void *lam_out, double *dL_dtau, double *dL_dbeta_in,
                            double *dL_de_in) {
  rlb_status s = check_reverse(h);
  if (s != RLB_OK) return s;
  if (!g_state_t || !lam_next || !lam_out || lam_next == lam_out)
    return fail(RLB_EINVAL, "adjoint buffers invalid");
  // the reader form goes to a library-owned block, then is gathered into lam_out
  if (!h->d_scratch) RLB_HIP(hipMalloc(&h->d_scratch, (size_t)Q * h->g.qs * h->lam_elem));
  auto launch = [&]() -> rlb_status {
    RLB_DISPATCH(h, launch_adjoint, h, g_state_t, lam_next, true, h->d_scratch);
  };
  s = launch();
  if (s == RLB_OK) s = launch_lam_gather(h, h->d_scratch, lam_out);
  if (s != RLB_OK) return s;
  if (dL_dtau || dL_dbeta_in || dL_de_in) return flush_adjoint(h, dL_dtau, dL_dbeta_in, dL_de_in);
  return RLB_OK;
}

rlb_status rlb_adjoint_segment(rlb_solver *h, const void *g_first, const void *g_seq,
                               int64_t seq_stride, int32_t n, void *lam_a, void *lam_b,
                               int32_t flags, void **lam_result) {
  rlb_status s = check_reverse(h);
  if (s != RLB_OK) return s;
  const bool in_reader = (flags & RLB_LAM_IN_READER) != 0;
  const bool out_reader = (flags & RLB_LAM_OUT_READER) != 0;
  const int blocks = g_first ? n - 1 : n;  // states read from g_seq
  if (n < 0 || !lam_a || !lam_b || lam_a == lam_b || !lam_result || seq_stride < 0 ||
      (blocks > 0 && !g_seq) || (flags & ~(RLB_LAM_IN_READER | RLB_LAM_OUT_READER)))
    return fail(RLB_EINVAL, "adjoint segment arguments invalid");
  if (n == 0 && out_reader && !in_reader)
    return fail(RLB_EINVAL, "a natural lambda has no reader form without a reverse step");
  const int64_t need = (int64_t)Q * h->g.qs * (int64_t)h->elem;
  if (blocks > 1 && seq_stride < need) return fail(RLB_EINVAL, "seq_stride below one g block");
  // steps ping-pong between lam_a and lam_b; a final gather (natural output)
  // writes the buffer not holding the last reader form
  const int writes = n + ((n > 0 || in_reader) && !out_reader ? 1 : 0);
  *lam_result = writes % 2 == 0 ? lam_a : lam_b;
  auto body = [&]() -> rlb_status {
    void *cur = lam_a, *nxt = lam_b;
    bool reader = in_reader;
    for (int j = n - 1; j >= 0; --j) {
      const void *S = g_first ? (j == 0 ? g_first
                                        : (const char *)g_seq + (size_t)(j - 1) * (size_t)seq_stride)
                              : (const char *)g_seq + (size_t)j * (size_t)seq_stride;
      auto launch = [&]() -> rlb_status {
        RLB_DISPATCH(h, launch_adjoint, h, S, (const void *)cur, !reader, nxt);
      };
      rlb_status st = launch();
      if (st != RLB_OK) return st;
      std::swap(cur, nxt);
      reader = true;
    }
    if (reader && !out_reader) return launch_lam_gather(h, cur, nxt);
    return RLB_OK;
  };
  if (n < kGraphMin) return body();
  // every captured step accumulates onto the pending partials: start them at zero
  if (!h->rev_pending) {
    s = zero_reverse_partials(h);
    if (s != RLB_OK) return s;
  }
  return run_graph(h, 3, g_seq, lam_a, lam_b, g_first, seq_stride, n, flags, body);
}

rlb_status rlb_adjoint_sweep(rlb_solver *h, const void *g_seq, int64_t seq_stride, int32_t n,
                             void *lam_a, void *lam_b, void **lam_result) {
  return rlb_adjoint_segment(h, nullptr, g_seq, seq_stride, n, lam_a, lam_b, 0, lam_result);
}

rlb_status rlb_lam_gather(rlb_solver *h, const void *lam_reader, void *lam_out) {
  rlb_status s = check_reverse(h);
  if (s != RLB_OK) return s;
  if (!lam_reader || !lam_out || lam_reader == lam_out)
    return fail(RLB_EINVAL, "lambda buffers invalid");
  return launch_lam_gather(h, lam_reader, lam_out);
}

rlb_status rlb_adjoint_flush(rlb_solver *h, double *dL_dtau, double *dL_dbeta_in,
                             double *dL_de_in) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  return flush_adjoint(h, dL_dtau, dL_dbeta_in, dL_de_in);
}

rlb_status rlb_advance_g(rlb_solver *h, const void *g_src, void *g_dst, void *g_tmp, int32_t n) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace) return fail(RLB_EINVAL, "the g-only and reverse entry points need the two-buffer layout (inplace = 0)");
  if (h->ph.eta_s > 0.0)
    return fail(RLB_EINVAL, "g-only steps and reverse steps are unavailable while eta/s is held");
  if (n < 0 || !g_src || !g_dst || g_src == g_dst || (n > 1 && (!g_tmp || g_tmp == g_src ||
                                                                 g_tmp == g_dst)))
    return fail(RLB_EINVAL, "advance arguments invalid");
  if (n == 0) {
    RLB_HIP(hipMemcpyAsync(g_dst, g_src, (size_t)Q * h->g.qs * h->elem,
                           hipMemcpyDeviceToDevice, h->stream));
    return RLB_OK;
  }
  auto body = [&]() -> rlb_status {
    const void *cur = g_src;
    for (int i = 0; i < n; ++i) {
      void *next = ((n - 1 - i) % 2 == 0) ? g_dst : g_tmp;  // the last step lands in g_dst
      auto launch = [&]() -> rlb_status { RLB_DISPATCH(h, launch_step_g, h, cur, next); };
      rlb_status s = launch();
      if (s != RLB_OK) return s;
      cur = next;
    }
    return RLB_OK;
  };
  if (n < kGraphMin) return body();
  return run_graph(h, 1, g_src, g_dst, g_tmp, nullptr, 0, n, 0, body);
}

rlb_status rlb_trajectory_g(rlb_solver *h, void *g_seq, int64_t seq_stride, int32_t n) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace) return fail(RLB_EINVAL, "the g-only and reverse entry points need the two-buffer layout (inplace = 0)");
  if (h->ph.eta_s > 0.0)
    return fail(RLB_EINVAL, "g-only steps and reverse steps are unavailable while eta/s is held");
  const int64_t need = (int64_t)Q * h->g.qs * (int64_t)h->elem;
  if (n < 1 || !g_seq || seq_stride < need) return fail(RLB_EINVAL, "trajectory arguments invalid");
  auto body = [&]() -> rlb_status {
    for (int j = 1; j < n; ++j) {
      const void *src = (const char *)g_seq + (size_t)(j - 1) * (size_t)seq_stride;
      void *dst = (char *)g_seq + (size_t)j * (size_t)seq_stride;
      auto launch = [&]() -> rlb_status { RLB_DISPATCH(h, launch_step_g, h, src, dst); };
      rlb_status s = launch();
      if (s != RLB_OK) return s;
    }
    return RLB_OK;
  };
  if (n - 1 < kGraphMin) return body();
  return run_graph(h, 2, g_seq, nullptr, nullptr, nullptr, seq_stride, n, 0, body);
}

rlb_status rlb_moments_adjoint(rlb_solver *h, const void *g_state_T, const double *dL_de,
                               const double *dL_dbeta, void *lam_T) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace) return fail(RLB_EINVAL, "the g-only and reverse entry points need the two-buffer layout (inplace = 0)");
  if (!g_state_T || !dL_de || !dL_dbeta || !lam_T)
    return fail(RLB_EINVAL, "a required pointer is NULL");
  RLB_DISPATCH(h, launch_moments_adjoint, h, g_state_T, dL_de, dL_dbeta, lam_T);
}

rlb_status rlb_init_adjoint(rlb_solver *h, const double *e0, const double *beta0,
                            const void *lam_0, double *dL_de0, double *dL_dbeta0,
                            double *dL_dbeta_in, double *dL_de_in) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace) return fail(RLB_EINVAL, "the g-only and reverse entry points need the two-buffer layout (inplace = 0)");
  if (!e0 || !beta0 || !lam_0 || !dL_de0 || !dL_dbeta0)
    return fail(RLB_EINVAL, "a required pointer is NULL");
  RLB_DISPATCH(h, launch_init_adjoint, h, e0, beta0, lam_0, dL_de0, dL_dbeta0, dL_dbeta_in,
               dL_de_in);
}

rlb_status rlb_set_tau_field(rlb_solver *h, const double *tau_cell) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  RLB_HIP(hipStreamSynchronize(h->stream));
  drop_graphs(h);  // captured kernels hold the old relaxation arguments
  const long long cells = (long long)h->g.batch * h->g.per;
  if (!tau_cell) {
    RLB_HIP(hipStreamSynchronize(h->stream));
    if (h->d_omega_cell) (void)hipFree(h->d_omega_cell);
    if (h->d_dtau_cell) (void)hipFree(h->d_dtau_cell);
    h->d_omega_cell = h->d_dtau_cell = nullptr;
    h->ph.omega_cell = nullptr;
    h->ph.dtau_cell = nullptr;
    return RLB_OK;
  }
  if (!h->d_bad) RLB_HIP(hipMalloc(&h->d_bad, sizeof(unsigned long long)));
  double *om = nullptr;
  RLB_HIP(hipMalloc(&om, sizeof(double) * (size_t)cells));
  unsigned long long nbad = 0;
  hipError_t e = hipMemsetAsync(h->d_bad, 0, sizeof(unsigned long long), h->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_set_omega_cell, dim3(grid_blocks(h)), dim3(BLOCK), 0, h->stream, h->g,
                       h->ph, tau_cell, om, h->d_bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(&nbad, h->d_bad, sizeof(nbad), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipFree(om);
    return fail(RLB_EDEVICE, std::string("rlb_set_tau_field: ") + hipGetErrorString(e));
  }
  if (nbad > 0) {
    (void)hipFree(om);
    return fail(RLB_EINVAL, "tau field: " + std::to_string(nbad) +
                                " non-solid cells with tau not > 1/2 (field unchanged)");
  }
  if (h->d_omega_cell) (void)hipFree(h->d_omega_cell);
  h->d_omega_cell = om;
  h->ph.omega_cell = om;
  if (!h->d_dtau_cell) RLB_HIP(hipMalloc(&h->d_dtau_cell, sizeof(double) * (size_t)cells));
  RLB_HIP(hipMemsetAsync(h->d_dtau_cell, 0, sizeof(double) * (size_t)cells, h->stream));
  h->ph.dtau_cell = h->d_dtau_cell;
  return RLB_OK;
}

rlb_status rlb_hold_eta_over_s(rlb_solver *h, double eta_over_s, double d_G) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (!(eta_over_s >= 0.0) || !std::isfinite(eta_over_s) || !(d_G > 0.0) || !std::isfinite(d_G))
    return fail(RLB_EINVAL, "eta_over_s must be >= 0 and d_G > 0 (both finite)");
  if (h->ph.gen_eos && eta_over_s > 0.0)
    return fail(RLB_EINVAL, "transport quantities and the eta/s rule are defined for e = 3P (kappa = 1/3)");
  if (h->inplace && eta_over_s > 0.0)
    return fail(RLB_EINVAL, "holding eta/s is built for the two-buffer layout (inplace = 0)");
  if (eta_over_s != h->ph.eta_s || d_G != h->ph.d_G) {
    RLB_HIP(hipStreamSynchronize(h->stream));
    drop_graphs(h);
  }
  h->ph.eta_s = eta_over_s;
  h->ph.d_G = d_G;
  return RLB_OK;
}

rlb_status rlb_transport(rlb_solver *h, double d_G, double *T, double *s, double *eta,
                         double *eta_over_s) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (h->inplace && h->aa_phase != 0)
    return fail(RLB_EINVAL, "in-place layout after an odd number of steps: S_t is not stored");
  if (h->ph.gen_eos)
    return fail(RLB_EINVAL, "transport quantities and the eta/s rule are defined for e = 3P (kappa = 1/3)");
  if (!(d_G > 0.0) || !std::isfinite(d_G)) return fail(RLB_EINVAL, "d_G must be > 0");
  if (h->ph.eta_s > 0.0 && d_G != h->ph.d_G)
    return fail(RLB_EINVAL, "d_G differs from the one eta/s is held with");
  const double keep = h->ph.d_G;
  h->ph.d_G = d_G;
  auto launch = [&]() -> rlb_status {
    RLB_DISPATCH(h, launch_transport, h, T, s, eta, eta_over_s);
  };
  rlb_status st = launch();
  h->ph.d_G = keep;
  return st;
}

rlb_status rlb_adjoint_flush_tau_field(rlb_solver *h, double *dL_dtau_cell) {
  if (check_handle(h) != RLB_OK) return RLB_EINVAL;
  if (!h->d_dtau_cell) return fail(RLB_EINVAL, "no tau field is set");
  if (!dL_dtau_cell) return fail(RLB_EINVAL, "dL_dtau_cell is NULL");
  const long long cells = (long long)h->g.batch * h->g.per;
  hipLaunchKernelGGL(k_take_cell_grad, dim3((unsigned)((cells + BLOCK - 1) / BLOCK)), dim3(BLOCK),
                     0, h->stream, cells, h->d_dtau_cell, dL_dtau_cell);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

rlb_status rlb_destroy(rlb_solver *h) {
  if (!h) return RLB_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  free_solver(h);
  if (e != hipSuccess) return fail(RLB_EDEVICE, hipGetErrorString(e));
  return RLB_OK;
}

rlb_status rlb_encode16(int32_t storage, const float *src, void *dst, int64_t n, void *stream) {
  if ((storage != RLB_F16DEV && storage != RLB_BF16DEV) || n < 0 || (n > 0 && (!src || !dst)))
    return fail(RLB_EINVAL, "rlb_encode16: storage must be RLB_F16DEV or RLB_BF16DEV, n >= 0, "
                            "non-NULL buffers");
  if (n == 0) return RLB_OK;
  const long long want = (n + BLOCK - 1) / BLOCK;
  const unsigned blocks = (unsigned)std::min<long long>(want, 1 << 20);
  const hipStream_t st = (hipStream_t)stream;
  if (storage == RLB_F16DEV)
    hipLaunchKernelGGL(k_encode16<ST_F16DEV>, dim3(blocks), dim3(BLOCK), 0, st, src,
                       (_Float16 *)dst, (long long)n);
  else
    hipLaunchKernelGGL(k_encode16<ST_BF16DEV>, dim3(blocks), dim3(BLOCK), 0, st, src,
                       (uint16_t *)dst, (long long)n);
  RLB_HIP(hipGetLastError());
  return RLB_OK;
}

const char *rlb_status_string(rlb_status s) {
  switch (s) {
    case RLB_OK: return "ok";
    case RLB_EINVAL: return "invalid argument";
    case RLB_ENOMEM: return "out of memory";
    case RLB_EDEVICE: return "device error";
    case RLB_EUNPHYSICAL: return "unphysical state (no real inversion of the moments)";
  }
  return "unknown status";
}

const char *rlb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
