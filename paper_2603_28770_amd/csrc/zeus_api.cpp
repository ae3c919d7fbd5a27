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

#include "zeus_host.h"
#include "zeus_internal.h"

namespace zeus {
namespace host {

thread_local std::string g_last_error;

zeus_err fail(zeus_err e, const std::string &msg) {
  g_last_error = msg;
  return e;
}

zeus_err hip_fail(hipError_t e, const char *what) {
  return fail(ZEUS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

zeus_err check_problem(const zeus_problem *p, bool user) {
  if (!p) return fail(ZEUS_EINVAL, "problem is NULL");
  if (p->abi_version != ZEUS_ABI_VERSION) return fail(ZEUS_EINVAL, "abi_version mismatch");
  if (user) {
    if (p->objective != ZEUS_USER) return fail(ZEUS_EINVAL, "objective must be ZEUS_USER");
    if (p->lbfgs_m == 0 && p->dim > zeus::kHybridDim)
      return fail(ZEUS_EUNSUPPORTED, "user objectives need dim <= 208 with BFGS (L-BFGS: <= 256)");
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

}  // namespace host
}  // namespace zeus

using namespace zeus::host;

namespace zeus {

namespace {
struct Layout {
  size_t best, gx, best_store, gx_store, part_key, part_f, part_idx, part_x, x, v, px, pf, es, total;
};
Layout layout(int64_t n, int dim, int es_len) {
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
  l.es = es_len > 0 ? take(sizeof(int32_t) * (size_t)es_len) : SIZE_MAX;
  l.total = o;
  return l;
}
}  // namespace

size_t workspace_bytes(int64_t n, int dim, int es_len) { return layout(n, dim, es_len).total; }

Workspace carve_workspace(void *base, int64_t n, int dim, int es_len) {
  const Layout l = layout(n, dim, es_len);
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
  w.es = l.es == SIZE_MAX ? nullptr : reinterpret_cast<int32_t *>(p + l.es);
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

int zeus::host::context_device(const zeus_context *ctx) { return ctx->device; }

struct zeus_user_objective {
  int device = 0;
  zeus::UserKernels k{};
};

namespace zeus {
int user_compile(const char *arch, const char *source, UserKernels *out, std::string *log);
void user_release(UserKernels *k);
}  // namespace zeus

namespace zeus {
namespace host {

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
// Ints of early-stop state in a request's workspace (0 without early stop).
int es_len_of(const zeus_problem &p) {
  return p.required_converged > 0 ? zeus::es_ints(p.iter_bfgs) : 0;
}
size_t request_ws_bytes(const zeus_problem &p) {
  return zeus::workspace_bytes(p.n_starts, p.dim, es_len_of(p));
}
zeus::Workspace carve_request_ws(void *base, const zeus_problem &p) {
  return zeus::carve_workspace(base, p.n_starts, p.dim, es_len_of(p));
}

// Builds the launch group of requests that share objective, precision and
// lane counts (nothing is enqueued).
zeus_err build_group(const std::vector<Planned> &reqs, void *hdr_table, void *hslots,
                     hipStream_t stream, GroupRun *run, bool need_hslots) {
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
  g.early_stop = false;
  g.resident = nullptr;
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
    q.out_skips = reqs[r].dev.skips;
    q.out_resets = reqs[r].dev.resets;
    q.trace = q.trace_len ? reqs[r].dev.trace : nullptr;
    q.summary = reqs[r].dev.summary;
    q.start_offset = g.total_starts;
    q.block_offset = g.pso_grid;
    q.required_c = p.required_converged;
    if (p.required_converged > 0) g.early_stop = true;
    g.total_starts += p.n_starts;
    g.pso_grid += q.ws.pso_blocks;
    if (p.iter_pso > g.max_iter_pso) g.max_iter_pso = p.iter_pso;
  }
  if (g.method == 0 && g.g_bfgs == zeus::kWideLanes) {
    const int dmax = max_dim(reqs);
    g.wide_slots = zeus::wide_slots(g.total_starts);
    g.wide_cs = zeus::wide_cs(dmax);
    g.wide_slot_doubles = (int64_t)dmax * g.wide_cs;
    if (!hslots && need_hslots) return fail(ZEUS_EINVAL, "wide problem without H slots");
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
                      bool with_copies, bool with_swarm) {
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
    TraceRange tr("zeus.swarm");
    for (int t = 0; t <= g.max_iter_pso; ++t)
      if ((e = zeus::launch_pso(g, t)) != hipSuccess) return hip_fail(e, "swarm launch");
    if ((e = zeus::launch_pso_finish(g)) != hipSuccess) return hip_fail(e, "swarm best launch");
  }
  if (prof) (void)hipEventRecord(pend.ev[1], stream);
  {
    TraceRange tr("zeus.bfgs");
    if ((e = zeus::launch_bfgs(g)) != hipSuccess) return hip_fail(e, "BFGS launch");
    if (g.early_stop) {  // K*, then the rerun of the starts that went past it
      if ((e = zeus::launch_es_finish(g)) != hipSuccess) return hip_fail(e, "early-stop launch");
      if ((e = zeus::launch_bfgs(g)) != hipSuccess) return hip_fail(e, "BFGS launch");
    }
  }
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
    ctx->prof.bfgs_launches += g.early_stop ? 2 : 1;
    ctx->prof.reduce_launches += 1;
  }
  return ZEUS_OK;
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
  l.sk = o; o += out.skips ? align_up(4 * n) : 0;
  l.rs = o; o += out.resets ? align_up(4 * n) : 0;
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
  dev.skips = out.skips ? reinterpret_cast<int32_t *>(R + l.sk) : nullptr;
  dev.resets = out.resets ? reinterpret_cast<int32_t *>(R + l.rs) : nullptr;
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
               {out.skips, dev.skips, 4 * n},
               {out.resets, dev.resets, 4 * n},
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
  bool operator<(const GroupKey &o) const {
    if (objective != o.objective) return objective < o.objective;
    if (method != o.method) return method < o.method;
    if (precision != o.precision) return precision < o.precision;
    if (g_pso != o.g_pso) return g_pso < o.g_pso;
    return g_bfgs < o.g_bfgs;
  }
};

GroupKey key_of(const zeus_problem &p) {
  return GroupKey{p.objective, p.precision, method_of(p), zeus::pso_group_lanes(p.dim),
                  lanes_of(p)};
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
    const GroupKey k = key_of(problems[r]);
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
    b.ws_total += request_ws_bytes(problems[r]);
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
  const size_t ng = b.order.size();
  std::vector<std::vector<Planned>> plans(ng);
  std::vector<GroupRun> runs(ng);
  // Every group's request table first, all on the first stream: an upload
  // from pageable host memory holds the host until its stream has finished
  // the work queued before it, so an upload behind another group's kernels
  // would keep the host from queueing anything else meanwhile.
  for (size_t gi = 0; gi < ng; ++gi) {
    const std::vector<int32_t> &members = b.groups.at(b.order[gi]);
    std::vector<Planned> &plan = plans[gi];
    plan.resize(members.size());
    for (size_t k = 0; k < members.size(); ++k) {
      const int32_t r = members[k];
      plan[k].pb = &problems[r];
      plan[k].dev = carve_result(R + b.res_off[r], b.rl[r], outs[r]);
      plan[k].ws = carve_request_ws(Wb + b.ws_off[r], problems[r]);
    }
    void *hs = b.h_off[gi] == SIZE_MAX ? nullptr : Wb + b.h_off[gi];
    if ((e = build_group(plan, Wb + b.tab_off[gi], hs, streams[gi % streams.size()], &runs[gi])) !=
        ZEUS_OK)
      return e;
    if ((e = upload_group(runs[gi], streams[0])) != ZEUS_OK) return e;
  }
  hipError_t he = hipStreamSynchronize(streams[0]);
  if (he != hipSuccess) return hip_fail(he, "hipStreamSynchronize");
  for (size_t gi = 0; gi < ng; ++gi)
    if ((e = launch_group(ctx, runs[gi], plans[gi], true)) != ZEUS_OK) return e;
  // Then the copies, after every group's kernels: a copy into pageable host
  // memory also holds the host until its stream gets there.  Issued between
  // groups, the copies and uploads kept the next groups' kernels from being
  // queued, so the persistent kernels of different groups never overlapped
  // (the full uneven batch spent a fifth of its time with the device idle).
  for (size_t gi = 0; gi < ng; ++gi) {
    hipStream_t s = streams[gi % streams.size()];
    const std::vector<int32_t> &members = b.groups.at(b.order[gi]);
    for (size_t k = 0; k < members.size(); ++k)
      if ((e = copy_back(problems[members[k]], outs[members[k]], plans[gi][k].dev, s)) != ZEUS_OK)
        return e;
  }
  return ZEUS_OK;
}

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void Pool::reset(size_t size) {
  free_.clear();
  if (size) free_[0] = size;
}

bool Pool::alloc(size_t bytes, size_t *off) {
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

void Pool::release(size_t off, size_t bytes) {
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

size_t Pool::largest() const {
  size_t m = 0;
  for (auto &kv : free_) m = kv.second > m ? kv.second : m;
  return m;
}

size_t Pool::free_bytes() const {
  size_t t = 0;
  for (auto &kv : free_) t += kv.second;
  return t;
}


}  // namespace host
}  // namespace zeus

// A captured solve: the kernels of every launch group of a batch in one HIP
// graph, bound to a caller-owned workspace and device outputs.
struct zeus_plan {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
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
  *bytes = kHdrBytes + table_bytes(1) + request_ws_bytes(*problem) +
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
  const size_t ws_bytes = request_ws_bytes(pb);
  one[0].ws = carve_request_ws(base + kHdrBytes + table_bytes(1), pb);
  void *hslots = hslot_bytes(hslot_lanes(pb), pb.n_starts, pb.dim)
                     ? base + kHdrBytes + table_bytes(1) + ws_bytes
                     : nullptr;
  return enqueue_group(ctx, one, base, hslots, s);
}
}  // namespace

zeus_err zeus_minimize_async(zeus_context *ctx, const zeus_problem *problem, void *workspace,
                             size_t workspace_bytes, const zeus_result *out, void *stream) {
  TraceRange tr("zeus_minimize_async");
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
  TraceRange tr("zeus_minimize_async_static");
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
  TraceRange tr(user ? "zeus_minimize_user" : "zeus_minimize_batch");
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
  if (e != ZEUS_OK) {
    // groups queued before the failure may still be running: let them end
    // before the caller reuses (or the next call reallocates) the buffers
    for (hipStream_t st : streams) (void)hipStreamSynchronize(st);
    return e;
  }
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
  TraceRange tr("zeus_plan_create");
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
      members[gi][k].ws = carve_request_ws(Wb + b.ws_off[idx[k]], problems[idx[k]]);
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
  TraceRange tr("zeus_plan_launch");
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
