// zeus_api.cpp -- the C ABI declared in include/zeus.h: validation, device
// workspace planning, contexts, and the launch sequence of a solve or a batch:
//   table upload -> counter reset -> swarm sweeps -> swarm best -> BFGS ->
//   summary
// enqueued per launch group on one HIP stream with no host round trip in
// between (groups of a batch on up to four streams).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <new>
#include <string>
#include <vector>

#include "zeus_internal.h"

namespace {

thread_local std::string g_last_error;

zeus_err fail(zeus_err e, const std::string &msg) {
  g_last_error = msg;
  return e;
}

zeus_err hip_fail(hipError_t e, const char *what) {
  return fail(ZEUS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Argument checks shared by every entry point taking a problem.
zeus_err check_problem(const zeus_problem *p, bool user = false) {
  if (!p) return fail(ZEUS_EINVAL, "problem is NULL");
  if (p->abi_version != ZEUS_ABI_VERSION) return fail(ZEUS_EINVAL, "abi_version mismatch");
  if (user) {
    if (p->objective != ZEUS_USER) return fail(ZEUS_EINVAL, "objective must be ZEUS_USER");
    if (p->precision != ZEUS_FP64) return fail(ZEUS_EUNSUPPORTED, "user objectives run in FP64");
    if (p->lbfgs_m == 0 && p->dim > zeus::kMaxNarrowDim)
      return fail(ZEUS_EUNSUPPORTED, "user objectives need dim <= 64 with BFGS (L-BFGS: <= 256)");
  } else if (p->objective == ZEUS_USER) {
    return fail(ZEUS_EINVAL, "ZEUS_USER problems run through zeus_minimize_user");
  } else if (p->objective < ZEUS_ROSENBROCK || p->objective > ZEUS_QUARTIC) {
    return fail(ZEUS_EINVAL, "unknown objective");
  }
  if (p->dim < 1) return fail(ZEUS_EINVAL, "dim must be >= 1");
  if (p->objective == ZEUS_ROSENBROCK && p->dim < 2)
    return fail(ZEUS_EINVAL, "Rosenbrock needs dim >= 2");
  if (p->objective == ZEUS_GOLDSTEIN_PRICE && p->dim != 2)
    return fail(ZEUS_EINVAL, "Goldstein-Price needs dim == 2");
  if (p->precision != ZEUS_FP64 && p->precision != ZEUS_MIXED)
    return fail(ZEUS_EINVAL, "unknown precision");
  if (p->n_starts < 1) return fail(ZEUS_EINVAL, "n_starts must be >= 1");
  if (!std::isfinite(p->lower) || !std::isfinite(p->upper) || !(p->lower < p->upper))
    return fail(ZEUS_EINVAL, "need finite lower < upper");
  if (p->iter_pso < 0 || p->iter_bfgs < 0 || p->iter_ls < 1)
    return fail(ZEUS_EINVAL, "need iter_pso >= 0, iter_bfgs >= 0, iter_ls >= 1");
  if (p->lbfgs_m < 0) return fail(ZEUS_EINVAL, "lbfgs_m must be >= 0");
  if (p->lbfgs_m > zeus::kLbfgsMaxHistory)
    return fail(ZEUS_EUNSUPPORTED, "lbfgs_m above 8 is not built");
  if (!std::isfinite(p->w) || !std::isfinite(p->c1) || !std::isfinite(p->c2) ||
      !std::isfinite(p->v_half))
    return fail(ZEUS_EINVAL, "PSO coefficients must be finite");
  if (!std::isfinite(p->grad_tol) || !(p->grad_tol > 0.0))
    return fail(ZEUS_EINVAL, "grad_tol must be > 0");
  if (!(p->armijo_c > 0.0 && p->armijo_c < 1.0))
    return fail(ZEUS_EINVAL, "armijo_c must be in (0,1)");
  if (!(p->ls_shrink > 0.0 && p->ls_shrink < 1.0))
    return fail(ZEUS_EINVAL, "ls_shrink must be in (0,1)");
  if (p->required_converged < 0) return fail(ZEUS_EINVAL, "required_converged must be >= 0");
  if (p->dim > zeus::kMaxDim) return fail(ZEUS_EUNSUPPORTED, "dim > 256 is not built");
  return ZEUS_OK;
}

zeus_err check_result(const zeus_result *r, const zeus_problem *p) {
  if (!r) return fail(ZEUS_EINVAL, "result is NULL");
  if (!r->f || !r->x || !r->iters || !r->status || !r->summary)
    return fail(ZEUS_EINVAL, "result needs f, x, iters, status and summary");
  if (r->trace_len < 0) return fail(ZEUS_EINVAL, "trace_len must be >= 0");
  if (r->trace && r->trace_len == 0) return fail(ZEUS_EINVAL, "trace given with trace_len 0");
  (void)p;
  return ZEUS_OK;
}

struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

namespace zeus {

namespace {
struct Layout {
  size_t best, gx, best_store, gx_store, part_key, part_f, part_idx, part_x, x, v, px, pf, total;
};
Layout layout(int64_t n, int dim) {
  const size_t P = (size_t)pso_blocks(n, dim), N = (size_t)n, D = (size_t)dim;
  Layout l;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  l.best = take(sizeof(PsoBest));
  l.gx = take(sizeof(double) * D);
  l.best_store = take(2 * sizeof(PsoBest));
  l.gx_store = take(2 * sizeof(double) * D);
  l.part_key = take(2 * sizeof(double) * P);
  l.part_f = take(2 * sizeof(double) * P);
  l.part_idx = take(2 * sizeof(int64_t) * P);
  l.part_x = take(2 * sizeof(double) * P * D);
  l.x = take(sizeof(double) * N * D);
  l.v = take(sizeof(double) * N * D);
  l.px = take(sizeof(double) * N * D);
  l.pf = take(sizeof(double) * N);
  l.total = o;
  return l;
}
}  // namespace

size_t workspace_bytes(int64_t n, int dim) { return layout(n, dim).total; }

Workspace carve_workspace(void *base, int64_t n, int dim) {
  const Layout l = layout(n, dim);
  char *p = static_cast<char *>(base);
  Workspace w;
  w.best = reinterpret_cast<PsoBest *>(p + l.best);
  w.gx = reinterpret_cast<double *>(p + l.gx);
  w.best_store = reinterpret_cast<PsoBest *>(p + l.best_store);
  w.gx_store = reinterpret_cast<double *>(p + l.gx_store);
  w.part_key = reinterpret_cast<double *>(p + l.part_key);
  w.part_f = reinterpret_cast<double *>(p + l.part_f);
  w.part_idx = reinterpret_cast<int64_t *>(p + l.part_idx);
  w.part_x = reinterpret_cast<double *>(p + l.part_x);
  w.x = reinterpret_cast<double *>(p + l.x);
  w.v = reinterpret_cast<double *>(p + l.v);
  w.px = reinterpret_cast<double *>(p + l.px);
  w.pf = reinterpret_cast<double *>(p + l.pf);
  w.pso_blocks = pso_blocks(n, dim);
  return w;
}

}  // namespace zeus

// The workspace of zeus_minimize_async_static: a fixed device array, one copy
// on every GPU the library runs on.  Host code never uses the array's name as
// an address (on the host it is a stand-in, not device memory); it uses the
// per-device address that hipGetSymbolAddress returns at context creation.
static __device__ __align__(256) unsigned char scratch[ZEUS_STATIC_WORKSPACE_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // by device; nullptr until resolved

// Resolves this device's copy of `scratch` once (the device must be current).
zeus_err bind_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)device < g_scratch_ptr.size() && g_scratch_ptr[(size_t)device]) return ZEUS_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static workspace");
  if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign != 0)
    return fail(ZEUS_EHIP, "static workspace address is not 256-byte aligned");
  if (g_scratch_ptr.size() <= (size_t)device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  g_scratch_ptr[(size_t)device] = ptr;
  return ZEUS_OK;
}

void *scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (size_t)device < g_scratch_ptr.size() ? g_scratch_ptr[(size_t)device] : nullptr;
}
}  // namespace

struct zeus_context {
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  // device buffers cached for the blocking entry points
  void *ws = nullptr;
  size_t ws_cap = 0;
  void *res = nullptr;
  size_t res_cap = 0;
  // extra streams so that independent launch groups of a batch overlap
  std::vector<hipStream_t> aux;
  // profiling
  bool profiling = false;
  struct Pending {
    hipEvent_t ev[4];  // before the swarm, after the swarm, after BFGS, after summary
  };
  std::vector<Pending> pending;
  zeus_profile prof{};
  // the user objective of the call in progress (set under mu)
  const zeus::UserKernels *active_user = nullptr;
};

struct zeus_user_objective {
  int device = 0;
  zeus::UserKernels k{};
};

namespace zeus {
int user_compile(const char *arch, const char *source, UserKernels *out, std::string *log);
void user_release(UserKernels *k);
}  // namespace zeus

namespace {

constexpr size_t kHdrBytes = 256;  // BatchDev, padded

size_t table_bytes(int nreq) { return align_up(sizeof(zeus::ReqDev) * (size_t)nreq); }

zeus_err ensure(void **buf, size_t *cap, size_t need) {
  if (*cap >= need) return ZEUS_OK;
  if (*buf) {
    (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
  }
  hipError_t e = hipMalloc(buf, need);
  if (e != hipSuccess) {
    *buf = nullptr;
    return fail(ZEUS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  *cap = need;
  return ZEUS_OK;
}

zeus_err drain_profile(zeus_context *ctx) {
  for (auto &p : ctx->pending) {
    hipError_t e = hipEventSynchronize(p.ev[3]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float a = 0, b = 0, c = 0;
    (void)hipEventElapsedTime(&a, p.ev[0], p.ev[1]);
    (void)hipEventElapsedTime(&b, p.ev[1], p.ev[2]);
    (void)hipEventElapsedTime(&c, p.ev[2], p.ev[3]);
    ctx->prof.pso_ms += a;
    ctx->prof.bfgs_ms += b;
    ctx->prof.reduce_ms += c;
    for (auto &ev : p.ev) (void)hipEventDestroy(ev);
  }
  ctx->pending.clear();
  return ZEUS_OK;
}

// One request of a launch group: its problem, device outputs and workspace.
struct Planned {
  const zeus_problem *pb;
  zeus_result dev;          // device pointers
  zeus::Workspace ws;
};

int max_dim(const std::vector<Planned> &reqs) {
  int d = 0;
  for (const Planned &q : reqs) d = q.pb->dim > d ? q.pb->dim : d;
  return d;
}

// Device bytes of the H slots a group needs (0 unless its problems are wide).
size_t hslot_bytes(int g_bfgs, int64_t total_starts, int dmax) {
  return g_bfgs == zeus::kWideLanes ? align_up(zeus::wide_hslot_bytes(total_starts, dmax)) : 0;
}

// Method (0 BFGS, 1 L-BFGS) and lanes / coordinate slots per start of a problem.
int method_of(const zeus_problem &p) { return p.lbfgs_m > 0 ? 1 : 0; }
// Early stop runs BFGS in capped passes, the first of at most 16
// iterations, which favour the narrowest group (16 or more starts per
// wavefront); the tiling table is tuned on full solves.  Built-in objectives
// with early stop therefore take the smallest power of two >= max(dim, 4)
// (unless ZEUS_TILE_LANES forces a tiling): in the Rastrigin studies at
// d <= 2 this ran the runs 3 times faster than the table's 32 lanes.
int lanes_of(const zeus_problem &p) {
  if (method_of(p)) return zeus::lbfgs_slots(p.dim);
  if (p.required_converged > 0 && p.objective != ZEUS_USER && p.dim <= zeus::kMaxNarrowDim &&
      !std::getenv("ZEUS_TILE_LANES")) {
    int g = 4;
    while (g < p.dim) g <<= 1;
    return g;
  }
  return zeus::group_lanes(p.objective, p.precision, p.dim);
}
// Only BFGS above the narrow limit keeps H in device-memory slots.
int hslot_lanes(const zeus_problem &p) { return method_of(p) ? 0 : lanes_of(p); }

// A launch group ready to run: the kernels' view (Group) and the host copy of
// its request table.
struct GroupRun {
  zeus::Group g;
  std::vector<zeus::ReqDev> host;
};

// Builds the launch group of requests that share objective, precision and
// lane counts (nothing is enqueued).
zeus_err build_group(const std::vector<Planned> &reqs, void *hdr_table, void *hslots,
                     hipStream_t stream, GroupRun *run) {
  zeus::Group &g = run->g;
  std::vector<zeus::ReqDev> &host = run->host;
  const zeus_problem &p0 = *reqs[0].pb;
  g.objective = p0.objective;
  g.precision = p0.precision;
  g.g_pso = zeus::pso_group_lanes(p0.dim);
  g.method = method_of(p0);
  g.g_bfgs = lanes_of(p0);
  g.nreq = (int)reqs.size();
  g.max_iter_pso = 0;
  g.pso_grid = 0;
  g.total_starts = 0;
  g.hdr = static_cast<zeus::BatchDev *>(hdr_table);
  g.reqs = reinterpret_cast<const zeus::ReqDev *>(static_cast<char *>(hdr_table) + kHdrBytes);
  g.stream = stream;
  g.hslots = static_cast<double *>(hslots);
  g.wide_slots = 0;
  g.wide_cs = 0;
  g.wide_slot_doubles = 0;
  g.user = nullptr;
  host.assign(reqs.size(), zeus::ReqDev{});
  for (size_t r = 0; r < reqs.size(); ++r) {
    const zeus_problem &p = *reqs[r].pb;
    zeus::ReqDev &q = host[r];
    std::memset(&q, 0, sizeof(q));
    q.n = p.n_starts;
    q.d = p.dim;
    q.iter_pso = p.iter_pso;
    q.iter_bfgs = p.iter_bfgs;
    q.iter_ls = p.iter_ls;
    q.stop_status = ZEUS_ST_MAXITER;
    q.lbfgs_m = p.lbfgs_m;
    q.trace_len = reqs[r].dev.trace ? reqs[r].dev.trace_len : 0;
    q.lo = p.lower;
    q.hi = p.upper;
    q.vh = p.v_half > 0.0 ? p.v_half : (p.upper - p.lower);
    q.w = p.w;
    q.c1 = p.c1;
    q.c2 = p.c2;
    q.armijo_c = p.armijo_c;
    q.shrink = p.ls_shrink;
    q.tol = p.grad_tol;
    q.k0 = p.seed;
    q.k1 = p.request_id;
    q.ws = reqs[r].ws;
    q.out_f = reqs[r].dev.f;
    q.out_x = reqs[r].dev.x;
    q.out_iters = reqs[r].dev.iters;
    q.out_status = reqs[r].dev.status;
    q.out_ls = reqs[r].dev.ls_trials;
    q.trace = q.trace_len ? reqs[r].dev.trace : nullptr;
    q.summary = reqs[r].dev.summary;
    q.start_offset = g.total_starts;
    q.block_offset = g.pso_grid;
    g.total_starts += p.n_starts;
    g.pso_grid += q.ws.pso_blocks;
    if (p.iter_pso > g.max_iter_pso) g.max_iter_pso = p.iter_pso;
  }
  if (g.method == 0 && g.g_bfgs == zeus::kWideLanes) {
    const int dmax = max_dim(reqs);
    g.wide_slots = zeus::wide_slots(g.total_starts);
    g.wide_cs = zeus::wide_cs(dmax);
    g.wide_slot_doubles = (int64_t)dmax * g.wide_cs;
    if (!hslots) return fail(ZEUS_EINVAL, "wide problem without H slots");
  }
  return ZEUS_OK;
}

zeus_err upload_group(const GroupRun &run, hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(const_cast<zeus::ReqDev *>(run.g.reqs), run.host.data(),
                                sizeof(zeus::ReqDev) * run.host.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "request table upload");
  return ZEUS_OK;
}

// Enqueues the kernels of a group on g.stream: counter reset, swarm sweeps
// 0..max iter_pso, swarm finish, one BFGS launch over all its starts, one
// summary block per request, then (with_copies) the optional swarm-state
// copies.  The request table must already be on the device.
zeus_err enqueue_copies(const std::vector<Planned> &reqs, hipStream_t stream) {
  hipError_t e;
  for (const Planned &q : reqs) {
    const size_t nd = sizeof(double) * (size_t)q.pb->n_starts * q.pb->dim;
    const size_t n8 = sizeof(double) * (size_t)q.pb->n_starts;
    struct Copy {
      void *dst;
      const void *src;
      size_t bytes;
    } copies[] = {{q.dev.seeds, q.ws.x, nd}, {q.dev.pso_v, q.ws.v, nd}, {q.dev.pso_px, q.ws.px, nd},
                  {q.dev.pso_pf, q.ws.pf, n8}, {q.dev.pso_best_x, q.ws.gx, sizeof(double) * q.pb->dim}};
    for (auto &c : copies)
      if (c.dst && (e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
  }
  return ZEUS_OK;
}

// Enqueues the kernels of a group on g.stream: counter reset, (with_swarm)
// swarm sweeps 0..max iter_pso and the swarm best, one BFGS launch over all
// its starts, one summary block per request, then (with_copies) the optional
// swarm-state copies.  The request table must already be on the device.
zeus_err launch_group(zeus_context *ctx, const GroupRun &run, const std::vector<Planned> &reqs,
                      bool with_copies, bool with_swarm = true) {
  zeus::Group g = run.g;
  if (g.objective == ZEUS_USER) {
    g.user = ctx ? ctx->active_user : nullptr;
    if (!g.user) return fail(ZEUS_EINVAL, "ZEUS_USER problem without a compiled objective");
  }
  hipStream_t stream = g.stream;
  hipError_t e;
  zeus_context::Pending pend{};
  const bool prof = ctx && ctx->profiling;
  if (prof)
    for (auto &ev : pend.ev)
      if (hipEventCreate(&ev) != hipSuccess) return fail(ZEUS_EHIP, "hipEventCreate failed");
  if (prof) (void)hipEventRecord(pend.ev[0], stream);
  if ((e = zeus::launch_ws_init(g)) != hipSuccess) return hip_fail(e, "counter reset launch");
  if (with_swarm) {
    for (int t = 0; t <= g.max_iter_pso; ++t)
      if ((e = zeus::launch_pso(g, t)) != hipSuccess) return hip_fail(e, "swarm launch");
    if ((e = zeus::launch_pso_finish(g)) != hipSuccess) return hip_fail(e, "swarm best launch");
  }
  if (prof) (void)hipEventRecord(pend.ev[1], stream);
  if ((e = zeus::launch_bfgs(g)) != hipSuccess) return hip_fail(e, "BFGS launch");
  if (prof) (void)hipEventRecord(pend.ev[2], stream);
  if ((e = zeus::launch_summary(g)) != hipSuccess) return hip_fail(e, "summary launch");
  if (prof) (void)hipEventRecord(pend.ev[3], stream);
  if (with_copies) {
    zeus_err ce = enqueue_copies(reqs, stream);
    if (ce != ZEUS_OK) return ce;
  }
  if (prof) {
    ctx->pending.push_back(pend);
    ctx->prof.pso_launches += with_swarm ? 3 + g.max_iter_pso : 0;
    ctx->prof.bfgs_launches += 1;
    ctx->prof.reduce_launches += 1;
  }
  return ZEUS_OK;
}

// Alg. 10's early stop for one request (required_converged = c > 0), read
// iteration-synchronously: K* is the iteration at which the c-th start
// converges; every start still running at K* ends there with status STOPPED.
// The swarm runs once; BFGS then runs from its seeds with an iteration cap
// of 16, 64, ... (x4, at most iter_bfgs) until at least c starts have
// converged, and a last time with the cap at K* when K* is below the cap.
// Each pass is deterministic, so the result is the same as a run that stops
// every start at K*.  Synchronises `stream` between passes.
zeus_err run_required(zeus_context *ctx, const std::vector<Planned> &reqs, void *hdr_table,
                      void *hslots, hipStream_t stream) {
  const zeus_problem &p = *reqs[0].pb;
  const int64_t c = p.required_converged, n = p.n_starts;
  std::vector<int32_t> it((size_t)n), st((size_t)n);
  int cap = p.iter_bfgs < 16 ? p.iter_bfgs : 16;
  bool swarm = true, last = false;
  zeus_err e;
  for (;;) {
    GroupRun run;
    if ((e = build_group(reqs, hdr_table, hslots, stream, &run)) != ZEUS_OK) return e;
    run.host[0].iter_bfgs = cap;
    run.host[0].stop_status = cap < p.iter_bfgs ? ZEUS_ST_STOPPED : ZEUS_ST_MAXITER;
    if ((e = upload_group(run, stream)) != ZEUS_OK) return e;
    if ((e = launch_group(ctx, run, reqs, false, swarm)) != ZEUS_OK) return e;
    swarm = false;
    if (last) break;
    hipError_t he = hipMemcpyAsync(it.data(), reqs[0].dev.iters, 4 * (size_t)n, hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(st.data(), reqs[0].dev.status, 4 * (size_t)n, hipMemcpyDeviceToHost, stream);
    if (he == hipSuccess) he = hipStreamSynchronize(stream);
    if (he != hipSuccess) return hip_fail(he, "early-stop pass");
    std::vector<int32_t> conv;
    for (int64_t i = 0; i < n; ++i)
      if (st[(size_t)i] == ZEUS_ST_CONVERGED) conv.push_back(it[(size_t)i]);
    if ((int64_t)conv.size() >= c) {
      std::nth_element(conv.begin(), conv.begin() + (c - 1), conv.end());
      const int kstar = conv[(size_t)(c - 1)];
      if (kstar == cap) break;
      cap = kstar;
      last = true;
    } else if (cap >= p.iter_bfgs) {
      break;  // fewer than c starts converge within the budget: no early stop
    } else {
      cap = cap * 4 < p.iter_bfgs ? cap * 4 : p.iter_bfgs;
    }
  }
  return enqueue_copies(reqs, stream);
}

// Build, upload and launch one group on `stream`.
zeus_err enqueue_group(zeus_context *ctx, const std::vector<Planned> &reqs, void *hdr_table,
                       void *hslots, hipStream_t stream) {
  GroupRun run;
  zeus_err e = build_group(reqs, hdr_table, hslots, stream, &run);
  if (e == ZEUS_OK) e = upload_group(run, stream);
  if (e == ZEUS_OK) e = launch_group(ctx, run, reqs, true);
  return e;
}

// Device result layout of one request for the blocking entry points.
struct ResLayout {
  size_t f, x, it, st, ls, seed, v, px, pf, gx, tr, sum, total;
};

ResLayout res_layout(const zeus_problem &pb, const zeus_result &out) {
  const size_t n = (size_t)pb.n_starts, d = (size_t)pb.dim;
  const size_t tl = out.trace ? (size_t)out.trace_len : 0;
  ResLayout l;
  size_t o = 0;
  l.f = o; o += align_up(8 * n);
  l.x = o; o += align_up(8 * n * d);
  l.it = o; o += align_up(4 * n);
  l.st = o; o += align_up(4 * n);
  l.ls = o; o += out.ls_trials ? align_up(4 * n) : 0;
  l.seed = o; o += out.seeds ? align_up(8 * n * d) : 0;
  l.v = o; o += out.pso_v ? align_up(8 * n * d) : 0;
  l.px = o; o += out.pso_px ? align_up(8 * n * d) : 0;
  l.pf = o; o += out.pso_pf ? align_up(8 * n) : 0;
  l.gx = o; o += out.pso_best_x ? align_up(8 * d) : 0;
  l.tr = o; o += tl ? align_up(8 * n * tl * d) : 0;
  l.sum = o; o += align_up(sizeof(zeus_summary));
  l.total = o;
  return l;
}

zeus_result carve_result(char *R, const ResLayout &l, const zeus_result &out) {
  zeus_result dev{};
  dev.f = reinterpret_cast<double *>(R + l.f);
  dev.x = reinterpret_cast<double *>(R + l.x);
  dev.iters = reinterpret_cast<int32_t *>(R + l.it);
  dev.status = reinterpret_cast<int32_t *>(R + l.st);
  dev.ls_trials = out.ls_trials ? reinterpret_cast<int32_t *>(R + l.ls) : nullptr;
  dev.seeds = out.seeds ? reinterpret_cast<double *>(R + l.seed) : nullptr;
  dev.pso_v = out.pso_v ? reinterpret_cast<double *>(R + l.v) : nullptr;
  dev.pso_px = out.pso_px ? reinterpret_cast<double *>(R + l.px) : nullptr;
  dev.pso_pf = out.pso_pf ? reinterpret_cast<double *>(R + l.pf) : nullptr;
  dev.pso_best_x = out.pso_best_x ? reinterpret_cast<double *>(R + l.gx) : nullptr;
  dev.trace = out.trace && out.trace_len ? reinterpret_cast<double *>(R + l.tr) : nullptr;
  dev.trace_len = dev.trace ? out.trace_len : 0;
  dev.summary = reinterpret_cast<zeus_summary *>(R + l.sum);
  return dev;
}

zeus_err copy_back(const zeus_problem &pb, const zeus_result &out, const zeus_result &dev,
                   hipStream_t s) {
  const size_t n = (size_t)pb.n_starts, d = (size_t)pb.dim;
  const size_t tl = dev.trace ? (size_t)dev.trace_len : 0;
  struct Back {
    void *dst;
    const void *src;
    size_t bytes;
  } backs[] = {{out.f, dev.f, 8 * n},
               {out.x, dev.x, 8 * n * d},
               {out.iters, dev.iters, 4 * n},
               {out.status, dev.status, 4 * n},
               {out.ls_trials, dev.ls_trials, 4 * n},
               {out.seeds, dev.seeds, 8 * n * d},
               {out.pso_v, dev.pso_v, 8 * n * d},
               {out.pso_px, dev.pso_px, 8 * n * d},
               {out.pso_pf, dev.pso_pf, 8 * n},
               {out.pso_best_x, dev.pso_best_x, 8 * d},
               {out.trace, dev.trace, 8 * n * tl * d},
               {out.summary, dev.summary, sizeof(zeus_summary)}};
  for (auto &b : backs)
    if (b.dst && b.src && b.bytes) {
      hipError_t e = hipMemcpyAsync(b.dst, b.src, b.bytes, hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync D2H");
    }
  return ZEUS_OK;
}

// Launch groups of a batch: requests that share objective, precision and
// lane counts run in one group.
struct GroupKey {
  int objective, precision, method, g_pso, g_bfgs;
  int64_t solo;  // > 0: a request with early stop, in a group of its own
  bool operator<(const GroupKey &o) const {
    if (solo != o.solo) return solo < o.solo;
    if (objective != o.objective) return objective < o.objective;
    if (method != o.method) return method < o.method;
    if (precision != o.precision) return precision < o.precision;
    if (g_pso != o.g_pso) return g_pso < o.g_pso;
    return g_bfgs < o.g_bfgs;
  }
};

GroupKey key_of(const zeus_problem &p, int32_t index) {
  return GroupKey{p.objective, p.precision, method_of(p), zeus::pso_group_lanes(p.dim),
                  lanes_of(p), p.required_converged > 0 ? (int64_t)index + 1 : 0};
}

// Device memory plan of a batch: result arrays of every request, then the
// swarm workspaces, then per launch group its header, request table and H
// slots.  Offsets are relative to two bases (results, workspace).
struct BatchPlan {
  std::map<GroupKey, std::vector<int32_t>> groups;
  std::vector<GroupKey> order;  // groups in the order of their first request
  std::vector<ResLayout> rl;
  std::vector<size_t> res_off, ws_off, tab_off, h_off;
  size_t res_total = 0, ws_total = 0;
};

BatchPlan plan_batch(const zeus_problem *problems, const zeus_result *outs, int32_t n) {
  BatchPlan b;
  for (int32_t r = 0; r < n; ++r) {
    const GroupKey k = key_of(problems[r], r);
    auto it = b.groups.find(k);
    if (it == b.groups.end()) b.order.push_back(k);
    b.groups[k].push_back(r);
  }
  b.rl.resize(n);
  b.res_off.resize(n);
  b.ws_off.resize(n);
  for (int32_t r = 0; r < n; ++r) {
    b.rl[r] = res_layout(problems[r], outs[r]);
    b.res_off[r] = b.res_total;
    b.res_total += b.rl[r].total;
    b.ws_off[r] = b.ws_total;
    b.ws_total += zeus::workspace_bytes(problems[r].n_starts, problems[r].dim);
  }
  b.tab_off.resize(b.order.size());
  b.h_off.resize(b.order.size());
  for (size_t gi = 0; gi < b.order.size(); ++gi) {
    const std::vector<int32_t> &members = b.groups[b.order[gi]];
    b.tab_off[gi] = b.ws_total;
    b.ws_total += kHdrBytes + table_bytes((int)members.size());
    int64_t starts = 0;
    int dmax = 0;
    for (int32_t r : members) {
      starts += problems[r].n_starts;
      dmax = problems[r].dim > dmax ? problems[r].dim : dmax;
    }
    const size_t hb = hslot_bytes(b.order[gi].method ? 0 : b.order[gi].g_bfgs, starts, dmax);
    b.h_off[gi] = hb ? b.ws_total : SIZE_MAX;
    b.ws_total += hb;
  }
  return b;
}

// Enqueues every launch group of a planned batch (group gi on
// streams[gi % streams.size()]) followed by the copies of its results into
// the host arrays of outs.
zeus_err enqueue_batch(zeus_context *ctx, const BatchPlan &b, const zeus_problem *problems,
                       const zeus_result *outs, void *res_base, void *ws_base,
                       const std::vector<hipStream_t> &streams) {
  char *R = static_cast<char *>(res_base), *Wb = static_cast<char *>(ws_base);
  zeus_err e;
  for (size_t gi = 0; gi < b.order.size(); ++gi) {
    hipStream_t s = streams[gi % streams.size()];
    const std::vector<int32_t> &members = b.groups.at(b.order[gi]);
    std::vector<Planned> plan(members.size());
    for (size_t k = 0; k < members.size(); ++k) {
      const int32_t r = members[k];
      plan[k].pb = &problems[r];
      plan[k].dev = carve_result(R + b.res_off[r], b.rl[r], outs[r]);
      plan[k].ws = zeus::carve_workspace(Wb + b.ws_off[r], problems[r].n_starts, problems[r].dim);
    }
    void *hs = b.h_off[gi] == SIZE_MAX ? nullptr : Wb + b.h_off[gi];
    if (b.order[gi].solo > 0)
      e = run_required(ctx, plan, Wb + b.tab_off[gi], hs, s);
    else
      e = enqueue_group(ctx, plan, Wb + b.tab_off[gi], hs, s);
    if (e != ZEUS_OK) return e;
    for (size_t k = 0; k < members.size(); ++k)
      if ((e = copy_back(problems[members[k]], outs[members[k]], plan[k].dev, s)) != ZEUS_OK)
        return e;
  }
  return ZEUS_OK;
}

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) of one device allocation.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto &kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> size
};

enum TicketState { kQueued, kRunning, kDone, kCancelled, kFailed };

struct Ticket {
  zeus_problem pb;
  zeus_result out;
  size_t bytes = 0;  // footprint of the request alone
  TicketState state = kQueued;
  zeus_err err = ZEUS_OK;
  std::string msg;
  zeus_request_times times{};
};

size_t footprint(const BatchPlan &b) { return align_up(b.res_total) + align_up(b.ws_total); }

}  // namespace

// A captured solve: the kernels of every launch group of a batch in one HIP
// graph, bound to a caller-owned workspace and device outputs.
struct zeus_plan {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

constexpr int kServerSlots = 4;       // batches in flight, one worker thread each
constexpr int kServerMaxBatch = 512;  // requests per batch

struct zeus_server {
  zeus_context *ctx = nullptr;
  int device = 0;
  void *mem = nullptr;
  size_t budget = 0;
  Pool pool;
  hipStream_t streams[kServerSlots] = {};
  std::mutex mu;
  std::condition_variable cv;        // workers: new requests or freed memory
  std::condition_variable done_cv;   // waiters: a ticket changed state
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_id = 1;
  bool stopping = false;
  std::vector<std::thread> workers;

  // Takes the longest prefix of the queue whose batch fits in the largest
  // free piece of the budget (lock held).  Returns false if the queue is
  // empty or its head does not fit now.
  bool take_batch(std::vector<uint64_t> &ids, std::vector<zeus_problem> &pbs,
                  std::vector<zeus_result> &outs, BatchPlan &plan, size_t &off, size_t &need) {
    const size_t room = pool.largest();
    ids.clear();
    pbs.clear();
    outs.clear();
    need = 0;
    for (uint64_t id : queue) {
      if ((int)ids.size() == kServerMaxBatch) break;
      const Ticket &t = tickets.at(id);
      pbs.push_back(t.pb);
      outs.push_back(t.out);
      BatchPlan trial = plan_batch(pbs.data(), outs.data(), (int32_t)pbs.size());
      const size_t f = footprint(trial);
      if (f > room) {
        pbs.pop_back();
        outs.pop_back();
        break;
      }
      ids.push_back(id);
      plan = std::move(trial);
      need = f;
    }
    if (ids.empty()) return false;
    for (size_t k = 0; k < ids.size(); ++k) queue.pop_front();
    (void)pool.alloc(need, &off);
    const uint64_t t0 = now_ns();
    for (uint64_t id : ids) {
      Ticket &t = tickets.at(id);
      t.state = kRunning;
      t.times.t_admit_ns = t0;
    }
    return true;
  }

  void work(int slot) {
    (void)hipSetDevice(device);
    std::vector<uint64_t> ids;
    std::vector<zeus_problem> pbs;
    std::vector<zeus_result> outs;
    BatchPlan plan;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      if (stopping && queue.empty()) break;
      size_t off = 0, need = 0;
      if (!take_batch(ids, pbs, outs, plan, off, need)) {
        cv.wait(lk);
        continue;
      }
      lk.unlock();
      // enqueue the batch and its copies into the callers' arrays, then wait
      char *base = static_cast<char *>(mem) + off;
      std::vector<hipStream_t> st{streams[slot]};
      zeus_err e = enqueue_batch(nullptr, plan, pbs.data(), outs.data(), base,
                                 base + align_up(plan.res_total), st);
      std::string msg = e != ZEUS_OK ? g_last_error : std::string();
      hipError_t he = hipStreamSynchronize(streams[slot]);
      if (e == ZEUS_OK && he != hipSuccess) {
        e = ZEUS_EHIP;
        msg = std::string("hipStreamSynchronize: ") + hipGetErrorString(he);
      }
      const uint64_t t1 = now_ns();
      lk.lock();
      for (uint64_t id : ids) {
        Ticket &t = tickets.at(id);
        t.state = e == ZEUS_OK ? kDone : kFailed;
        t.err = e;
        t.msg = msg;
        t.times.t_done_ns = t1;
      }
      pool.release(off, need);
      done_cv.notify_all();
      cv.notify_all();  // freed memory may let a waiting head in
    }
  }
};

extern "C" {

uint32_t zeus_abi_version(void) { return ZEUS_ABI_VERSION; }

const char *zeus_version(void) { return "zeus-mi355x 0.2.0 (gfx950)"; }

const char *zeus_last_error(void) { return g_last_error.c_str(); }

zeus_err zeus_validate(const zeus_problem *problem) {
  g_last_error.clear();
  return check_problem(problem);
}

zeus_err zeus_workspace_bytes(const zeus_problem *problem, size_t *bytes) {
  g_last_error.clear();
  if (!bytes) return fail(ZEUS_EINVAL, "bytes is NULL");
  zeus_err e = check_problem(problem);
  if (e != ZEUS_OK) return e;
  *bytes = kHdrBytes + table_bytes(1) + zeus::workspace_bytes(problem->n_starts, problem->dim) +
           hslot_bytes(hslot_lanes(*problem), problem->n_starts, problem->dim);
  return ZEUS_OK;
}

zeus_err zeus_context_create(int device, zeus_context **out) {
  g_last_error.clear();
  if (!out) return fail(ZEUS_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= count) return fail(ZEUS_EINVAL, "no such device");
  zeus_context *ctx = new (std::nothrow) zeus_context;
  if (!ctx) return fail(ZEUS_ENOMEM, "context allocation failed");
  ctx->device = device;
  DeviceGuard g(device);
  if (g.err != hipSuccess) {
    delete ctx;
    return hip_fail(g.err, "hipSetDevice");
  }
  e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete ctx;
    return hip_fail(e, "hipStreamCreate");
  }
  zeus_err se = bind_scratch(device);
  if (se != ZEUS_OK) {
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return se;
  }
  *out = ctx;
  return ZEUS_OK;
}

zeus_err zeus_context_destroy(zeus_context *ctx) {
  g_last_error.clear();
  if (!ctx) return ZEUS_OK;
  {
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipStream_t s : ctx->aux) (void)hipStreamSynchronize(s);
    (void)drain_profile(ctx);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->res) (void)hipFree(ctx->res);
    for (hipStream_t s : ctx->aux) (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
  return ZEUS_OK;
}

zeus_err zeus_context_set_profiling(zeus_context *ctx, int enabled) {
  g_last_error.clear();
  if (!ctx) return fail(ZEUS_EINVAL, "ctx is NULL");
  DeviceGuard g(ctx->device);
  std::lock_guard<std::mutex> lk(ctx->mu);
  zeus_err e = drain_profile(ctx);
  ctx->profiling = enabled != 0;
  ctx->prof = zeus_profile{};
  return e;
}

zeus_err zeus_context_get_profile(zeus_context *ctx, zeus_profile *out) {
  g_last_error.clear();
  if (!ctx || !out) return fail(ZEUS_EINVAL, "NULL argument");
  DeviceGuard g(ctx->device);
  std::lock_guard<std::mutex> lk(ctx->mu);
  zeus_err e = drain_profile(ctx);
  *out = ctx->prof;
  return e;
}

namespace {
// Argument checks of the asynchronous entry points; *need receives the
// workspace bytes of the problem.
zeus_err check_async(zeus_context *ctx, const zeus_problem *problem, const zeus_result *out,
                     size_t *need) {
  if (!ctx) return fail(ZEUS_EINVAL, "ctx is NULL");
  zeus_err e = check_problem(problem);
  if (e != ZEUS_OK) return e;
  if ((e = check_result(out, problem)) != ZEUS_OK) return e;
  if (problem->required_converged > 0)
    return fail(ZEUS_EUNSUPPORTED, "early stopping needs zeus_minimize, zeus_minimize_batch or a server");
  return zeus_workspace_bytes(problem, need);
}

// Enqueues one solve on `stream` in the workspace at `workspace` (256-byte
// aligned, at least zeus_workspace_bytes()); the device is current.
zeus_err enqueue_async(zeus_context *ctx, const zeus_problem &pb, void *workspace,
                       const zeus_result *out, hipStream_t s) {
  char *base = static_cast<char *>(workspace);
  std::vector<Planned> one(1);
  one[0].pb = &pb;
  one[0].dev = *out;
  if (!one[0].dev.trace || one[0].dev.trace_len == 0) {
    one[0].dev.trace = nullptr;
    one[0].dev.trace_len = 0;
  }
  const size_t ws_bytes = zeus::workspace_bytes(pb.n_starts, pb.dim);
  one[0].ws = zeus::carve_workspace(base + kHdrBytes + table_bytes(1), pb.n_starts, pb.dim);
  void *hslots = hslot_bytes(hslot_lanes(pb), pb.n_starts, pb.dim)
                     ? base + kHdrBytes + table_bytes(1) + ws_bytes
                     : nullptr;
  return enqueue_group(ctx, one, base, hslots, s);
}
}  // namespace

zeus_err zeus_minimize_async(zeus_context *ctx, const zeus_problem *problem, void *workspace,
                             size_t workspace_bytes, const zeus_result *out, void *stream) {
  g_last_error.clear();
  size_t need = 0;
  zeus_err e = check_async(ctx, problem, out, &need);
  if (e != ZEUS_OK) return e;
  if (!workspace || workspace_bytes < need)
    return fail(ZEUS_EINVAL, "workspace missing or smaller than zeus_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(ZEUS_EINVAL, "workspace must be 256-byte aligned");
  const zeus_problem pb = *problem;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  std::lock_guard<std::mutex> lk(ctx->mu);
  return enqueue_async(ctx, pb, workspace, out,
                       stream ? static_cast<hipStream_t>(stream) : ctx->stream);
}

zeus_err zeus_minimize_async_static(zeus_context *ctx, const zeus_problem *problem,
                                    const zeus_result *out, void *stream) {
  g_last_error.clear();
  size_t need = 0;
  zeus_err e = check_async(ctx, problem, out, &need);
  if (e != ZEUS_OK) return e;
  if (need > ZEUS_STATIC_WORKSPACE_BYTES)
    return fail(ZEUS_ENOMEM, "problem needs " + std::to_string(need) +
                                 " bytes of workspace; the static workspace holds " +
                                 std::to_string(ZEUS_STATIC_WORKSPACE_BYTES));
  void *ws = scratch_of(ctx->device);
  if (!ws) return fail(ZEUS_EHIP, "static workspace not resolved on this device");
  const zeus_problem pb = *problem;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  std::lock_guard<std::mutex> lk(ctx->mu);
  return enqueue_async(ctx, pb, ws, out, stream ? static_cast<hipStream_t>(stream) : ctx->stream);
}

zeus_err zeus_minimize(zeus_context *ctx, const zeus_problem *problem, const zeus_result *out) {
  return zeus_minimize_batch(ctx, problem, 1, out);
}

namespace {
// zeus_minimize_batch, and zeus_minimize_user with `user` set.
zeus_err minimize_batch(zeus_context *ctx, const zeus_problem *problems, int32_t n,
                        const zeus_result *outs, const zeus_user_objective *user) {
  g_last_error.clear();
  if (!ctx) return fail(ZEUS_EINVAL, "ctx is NULL");
  if (n < 1 || !problems || !outs) return fail(ZEUS_EINVAL, "need n >= 1 problems and results");
  if (user && user->device != ctx->device)
    return fail(ZEUS_EINVAL, "the objective was compiled for another device");
  for (int32_t r = 0; r < n; ++r) {
    zeus_err e = check_problem(&problems[r], user != nullptr);
    if (e == ZEUS_OK) e = check_result(&outs[r], &problems[r]);
    if (e != ZEUS_OK) return fail(e, "request " + std::to_string(r) + ": " + g_last_error);
  }
  const BatchPlan plan = plan_batch(problems, outs, n);
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  std::lock_guard<std::mutex> lk(ctx->mu);
  zeus_err e;
  if ((e = ensure(&ctx->ws, &ctx->ws_cap, plan.ws_total)) != ZEUS_OK) return e;
  if ((e = ensure(&ctx->res, &ctx->res_cap, plan.res_total)) != ZEUS_OK) return e;
  // independent groups run on separate streams so that their kernels overlap
  const size_t want_streams = plan.order.size() < 4 ? plan.order.size() : 4;
  while (ctx->aux.size() + 1 < want_streams) {
    hipStream_t s;
    hipError_t he = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (he != hipSuccess) return hip_fail(he, "hipStreamCreate");
    ctx->aux.push_back(s);
  }
  std::vector<hipStream_t> streams{ctx->stream};
  for (size_t k = 0; k + 1 < want_streams; ++k) streams.push_back(ctx->aux[k]);
  ctx->active_user = user ? &user->k : nullptr;
  e = enqueue_batch(ctx, plan, problems, outs, ctx->res, ctx->ws, streams);
  ctx->active_user = nullptr;
  if (e != ZEUS_OK) return e;
  hipError_t he;
  for (hipStream_t st : streams)
    if ((he = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(he, "hipStreamSynchronize");
  return ZEUS_OK;
}
}  // namespace

zeus_err zeus_minimize_batch(zeus_context *ctx, const zeus_problem *problems, int32_t n,
                             const zeus_result *outs) {
  return minimize_batch(ctx, problems, n, outs, nullptr);
}

zeus_err zeus_minimize_user(zeus_context *ctx, const zeus_user_objective *obj,
                            const zeus_problem *problems, int32_t n, const zeus_result *outs) {
  if (!obj) {
    g_last_error.clear();
    return fail(ZEUS_EINVAL, "objective is NULL");
  }
  return minimize_batch(ctx, problems, n, outs, obj);
}

zeus_err zeus_objective_check(const char *source) {
  g_last_error.clear();
  if (!source) return fail(ZEUS_EINVAL, "source is NULL");
  std::string log;
  const int r = zeus::user_compile("gfx950", source, nullptr, &log);
  if (r == 1) return fail(ZEUS_EINVAL, "objective does not compile:\n" + log);
  if (r != 0) return fail(ZEUS_EHIP, log);
  return ZEUS_OK;
}

zeus_err zeus_objective_compile(zeus_context *ctx, const char *source, zeus_user_objective **out) {
  g_last_error.clear();
  if (!ctx || !source || !out) return fail(ZEUS_EINVAL, "NULL argument");
  *out = nullptr;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipDeviceProp_t prop;
  hipError_t he = hipGetDeviceProperties(&prop, ctx->device);
  if (he != hipSuccess) return hip_fail(he, "hipGetDeviceProperties");
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  auto *obj = new (std::nothrow) zeus_user_objective;
  if (!obj) return fail(ZEUS_ENOMEM, "allocation failed");
  obj->device = ctx->device;
  std::string log;
  const int r = zeus::user_compile(arch.c_str(), source, &obj->k, &log);
  if (r != 0) {
    delete obj;
    return fail(r == 1 ? ZEUS_EINVAL : ZEUS_EHIP,
                r == 1 ? "objective does not compile:\n" + log : log);
  }
  *out = obj;
  return ZEUS_OK;
}

zeus_err zeus_objective_destroy(zeus_user_objective *obj) {
  g_last_error.clear();
  if (!obj) return ZEUS_OK;
  {
    DeviceGuard dg(obj->device);
    zeus::user_release(&obj->k);
  }
  delete obj;
  return ZEUS_OK;
}


zeus_err zeus_server_create(zeus_context *ctx, size_t hbm_budget_bytes, zeus_server **out) {
  g_last_error.clear();
  if (!ctx || !out) return fail(ZEUS_EINVAL, "NULL argument");
  *out = nullptr;
  if (hbm_budget_bytes < ((size_t)1 << 20)) return fail(ZEUS_EINVAL, "budget below 1 MiB");
  auto *srv = new (std::nothrow) zeus_server;
  if (!srv) return fail(ZEUS_ENOMEM, "server allocation failed");
  srv->ctx = ctx;
  srv->device = ctx->device;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) {
    delete srv;
    return hip_fail(g.err, "hipSetDevice");
  }
  srv->budget = hbm_budget_bytes / kAlign * kAlign;
  hipError_t e = hipMalloc(&srv->mem, srv->budget);
  if (e != hipSuccess) {
    delete srv;
    return fail(ZEUS_ENOMEM, std::string("hipMalloc of the budget: ") + hipGetErrorString(e));
  }
  srv->pool.reset(srv->budget);
  for (auto &st : srv->streams) {
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) {
      for (auto &s2 : srv->streams)
        if (s2) (void)hipStreamDestroy(s2);
      (void)hipFree(srv->mem);
      delete srv;
      return hip_fail(e, "hipStreamCreate");
    }
  }
  for (int k = 0; k < kServerSlots; ++k) srv->workers.emplace_back([srv, k] { srv->work(k); });
  *out = srv;
  return ZEUS_OK;
}

zeus_err zeus_server_submit(zeus_server *srv, const zeus_problem *problem,
                            const zeus_result *host_out, uint64_t *ticket) {
  g_last_error.clear();
  if (!srv || !ticket) return fail(ZEUS_EINVAL, "NULL argument");
  zeus_err e = check_problem(problem);
  if (e == ZEUS_OK) e = check_result(host_out, problem);
  if (e != ZEUS_OK) return e;
  Ticket t;
  t.pb = *problem;
  t.out = *host_out;
  if (!t.out.trace || t.out.trace_len == 0) {
    t.out.trace = nullptr;
    t.out.trace_len = 0;
  }
  t.bytes = footprint(plan_batch(&t.pb, &t.out, 1));
  if (t.bytes > srv->budget)
    return fail(ZEUS_ENOMEM, "request needs " + std::to_string(t.bytes) +
                                 " bytes of device memory, more than the server's budget");
  t.times.t_submit_ns = now_ns();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stopping) return fail(ZEUS_ECANCELLED, "server is shutting down");
  const uint64_t id = srv->next_id++;
  srv->tickets.emplace(id, t);
  srv->queue.push_back(id);
  *ticket = id;
  srv->cv.notify_one();
  return ZEUS_OK;
}

zeus_err zeus_server_wait(zeus_server *srv, uint64_t ticket, int64_t timeout_ns,
                          zeus_request_times *times) {
  g_last_error.clear();
  if (!srv) return fail(ZEUS_EINVAL, "srv is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns > 0 ? timeout_ns : 0);
  for (;;) {
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(ZEUS_EINVAL, "unknown or released ticket");
    Ticket &t = it->second;
    if (t.state == kDone || t.state == kCancelled || t.state == kFailed) {
      if (times) *times = t.times;
      const TicketState st = t.state;
      const zeus_err err = t.err;
      const std::string msg = t.msg;
      srv->tickets.erase(it);
      if (st == kDone) return ZEUS_OK;
      if (st == kCancelled) return fail(ZEUS_ECANCELLED, "request was cancelled");
      return fail(err, msg);
    }
    if (timeout_ns == 0) return ZEUS_NOT_READY;
    if (timeout_ns < 0) {
      srv->done_cv.wait(lk);
    } else if (srv->done_cv.wait_until(lk, deadline) == std::cv_status::timeout) {
      auto again = srv->tickets.find(ticket);
      if (again != srv->tickets.end() && (again->second.state == kQueued || again->second.state == kRunning))
        return fail(ZEUS_ETIMEOUT, "timed out");
    }
  }
}

zeus_err zeus_server_cancel(zeus_server *srv, uint64_t ticket) {
  g_last_error.clear();
  if (!srv) return fail(ZEUS_EINVAL, "srv is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return fail(ZEUS_EINVAL, "unknown or released ticket");
  if (it->second.state != kQueued) {
    if (it->second.state == kRunning) {
      g_last_error = "request is running; wait for it";
      return ZEUS_NOT_READY;
    }
    return ZEUS_OK;  // already finished
  }
  for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
    if (*q == ticket) {
      srv->queue.erase(q);
      break;
    }
  it->second.state = kCancelled;
  srv->done_cv.notify_all();
  srv->cv.notify_one();
  return ZEUS_OK;
}

zeus_err zeus_server_destroy(zeus_server *srv) {
  g_last_error.clear();
  if (!srv) return ZEUS_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    for (uint64_t id : srv->queue) srv->tickets.at(id).state = kCancelled;
    srv->queue.clear();
    srv->cv.notify_all();
    srv->done_cv.notify_all();
  }
  for (auto &w : srv->workers) w.join();
  {
    DeviceGuard g(srv->device);
    for (auto &st : srv->streams) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    (void)hipFree(srv->mem);
  }
  delete srv;
  return ZEUS_OK;
}


zeus_err zeus_plan_workspace_bytes(const zeus_problem *problems, int32_t n, size_t *bytes) {
  g_last_error.clear();
  if (!problems || n < 1 || !bytes) return fail(ZEUS_EINVAL, "need n >= 1 problems and bytes");
  std::vector<zeus_result> none(n);
  for (int32_t r = 0; r < n; ++r) {
    zeus_err e = check_problem(&problems[r]);
    if (e != ZEUS_OK) return fail(e, "request " + std::to_string(r) + ": " + g_last_error);
  }
  *bytes = plan_batch(problems, none.data(), n).ws_total;
  return ZEUS_OK;
}

zeus_err zeus_plan_create(zeus_context *ctx, const zeus_problem *problems, int32_t n,
                          void *workspace, size_t workspace_bytes, const zeus_result *outs,
                          zeus_plan **out) {
  g_last_error.clear();
  if (!ctx || !out) return fail(ZEUS_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1 || !problems || !outs) return fail(ZEUS_EINVAL, "need n >= 1 problems and results");
  for (int32_t r = 0; r < n; ++r) {
    zeus_err e = check_problem(&problems[r]);
    if (e == ZEUS_OK) e = check_result(&outs[r], &problems[r]);
    if (e == ZEUS_OK && (outs[r].seeds || outs[r].pso_v || outs[r].pso_px || outs[r].pso_pf ||
                         outs[r].pso_best_x))
      e = fail(ZEUS_EINVAL, "swarm-state outputs are not available in a plan");
    if (e == ZEUS_OK && problems[r].required_converged > 0)
      e = fail(ZEUS_EUNSUPPORTED, "early stopping is not available in a plan");
    if (e != ZEUS_OK) return fail(e, "request " + std::to_string(r) + ": " + g_last_error);
  }
  std::vector<zeus_result> res(outs, outs + n);
  for (auto &r : res)
    if (!r.trace || r.trace_len == 0) {
      r.trace = nullptr;
      r.trace_len = 0;
    }
  const BatchPlan b = plan_batch(problems, res.data(), n);
  if (!workspace || workspace_bytes < b.ws_total)
    return fail(ZEUS_EINVAL, "workspace missing or smaller than zeus_plan_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(ZEUS_EINVAL, "workspace must be 256-byte aligned");
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  std::lock_guard<std::mutex> lk(ctx->mu);
  // build every group and upload its request table (outside the graph)
  char *Wb = static_cast<char *>(workspace);
  std::vector<std::vector<Planned>> members(b.order.size());
  std::vector<GroupRun> runs(b.order.size());
  zeus_err e;
  for (size_t gi = 0; gi < b.order.size(); ++gi) {
    const std::vector<int32_t> &idx = b.groups.at(b.order[gi]);
    members[gi].resize(idx.size());
    for (size_t k = 0; k < idx.size(); ++k) {
      members[gi][k].pb = &problems[idx[k]];
      members[gi][k].dev = res[idx[k]];
      members[gi][k].ws =
          zeus::carve_workspace(Wb + b.ws_off[idx[k]], problems[idx[k]].n_starts, problems[idx[k]].dim);
    }
    void *hs = b.h_off[gi] == SIZE_MAX ? nullptr : Wb + b.h_off[gi];
    if ((e = build_group(members[gi], Wb + b.tab_off[gi], hs, ctx->stream, &runs[gi])) != ZEUS_OK)
      return e;
    if ((e = upload_group(runs[gi], ctx->stream)) != ZEUS_OK) return e;
  }
  hipError_t he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return hip_fail(he, "hipStreamSynchronize");
  // capture: groups fork from the context's stream onto up to four streams
  const size_t nstreams = b.order.size() < 4 ? b.order.size() : 4;
  while (ctx->aux.size() + 1 < nstreams) {
    hipStream_t st;
    if ((he = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(he, "hipStreamCreate");
    ctx->aux.push_back(st);
  }
  std::vector<hipStream_t> streams{ctx->stream};
  for (size_t k = 0; k + 1 < nstreams; ++k) streams.push_back(ctx->aux[k]);
  std::vector<hipEvent_t> evs(nstreams + 1, nullptr);
  for (auto &ev : evs)
    if ((he = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
      for (auto &e2 : evs)
        if (e2) (void)hipEventDestroy(e2);
      return hip_fail(he, "hipEventCreate");
    }
  auto *plan = new (std::nothrow) zeus_plan;
  if (!plan) return fail(ZEUS_ENOMEM, "plan allocation failed");
  plan->device = ctx->device;
  zeus_err err = ZEUS_OK;
  he = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed);
  if (he == hipSuccess) {
    (void)hipEventRecord(evs[0], ctx->stream);
    for (size_t k = 1; k < nstreams; ++k) (void)hipStreamWaitEvent(streams[k], evs[0], 0);
    for (size_t gi = 0; gi < b.order.size() && err == ZEUS_OK; ++gi) {
      runs[gi].g.stream = streams[gi % nstreams];
      err = launch_group(nullptr, runs[gi], members[gi], false);
    }
    for (size_t k = 1; k < nstreams; ++k) {
      (void)hipEventRecord(evs[k], streams[k]);
      (void)hipStreamWaitEvent(ctx->stream, evs[k], 0);
    }
    hipError_t ce = hipStreamEndCapture(ctx->stream, &plan->graph);
    if (err == ZEUS_OK && ce != hipSuccess) err = hip_fail(ce, "hipStreamEndCapture");
  } else {
    err = hip_fail(he, "hipStreamBeginCapture");
  }
  for (auto &ev : evs) (void)hipEventDestroy(ev);
  if (err == ZEUS_OK && (he = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0)) != hipSuccess)
    err = hip_fail(he, "hipGraphInstantiate");
  if (err != ZEUS_OK) {
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return err;
  }
  *out = plan;
  return ZEUS_OK;
}

zeus_err zeus_plan_launch(zeus_plan *plan, void *stream) {
  g_last_error.clear();
  if (!plan) return fail(ZEUS_EINVAL, "plan is NULL");
  DeviceGuard dg(plan->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ZEUS_OK;
}

zeus_err zeus_plan_destroy(zeus_plan *plan) {
  g_last_error.clear();
  if (!plan) return ZEUS_OK;
  DeviceGuard dg(plan->device);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
  return ZEUS_OK;
}

}  // extern "C"
