// zeus_api.cpp -- the C ABI declared in include/zeus.h: validation, device
// workspace planning, contexts, and the launch sequence of one solve:
//   workspace init -> swarm init -> iter_pso swarm updates -> BFGS -> summary
// all enqueued on one HIP stream with no host round trip in between.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
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
zeus_err check_problem(const zeus_problem *p) {
  if (!p) return fail(ZEUS_EINVAL, "problem is NULL");
  if (p->abi_version != ZEUS_ABI_VERSION) return fail(ZEUS_EINVAL, "abi_version mismatch");
  if (p->objective < ZEUS_ROSENBROCK || p->objective > ZEUS_QUARTIC)
    return fail(ZEUS_EINVAL, "unknown objective");
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
  if (p->reserved0 != 0) return fail(ZEUS_EINVAL, "reserved0 must be 0");
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
  if (p->required_converged != 0)
    return fail(ZEUS_EUNSUPPORTED, "early stopping (required_converged > 0) is not built");
  if (p->dim > zeus::kMaxDim) return fail(ZEUS_EUNSUPPORTED, "dim > 64 is not built");
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
  size_t queue, best, gx, best_store, gx_store, part_key, part_f, part_idx, part_x, x, v, px,
      pf, total;
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
  l.queue = take(sizeof(uint64_t));
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
  w.queue = reinterpret_cast<uint64_t *>(p + l.queue);
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

struct zeus_context {
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  // device buffers cached for the blocking entry point
  void *ws = nullptr;
  size_t ws_cap = 0;
  void *res = nullptr;
  size_t res_cap = 0;
  // profiling
  bool profiling = false;
  struct Pending {
    hipEvent_t ev[4];  // before PSO, after PSO, after BFGS, after summary
  };
  std::vector<Pending> pending;
  zeus_profile prof{};
};

namespace {

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

// Enqueues the whole solve.  `out` holds device pointers.
zeus_err enqueue_solve(zeus_context *ctx, const zeus_problem *pb, void *ws_base,
                       const zeus_result *out, hipStream_t stream) {
  zeus::Launch L;
  L.pb = pb;
  L.out = out;
  L.ws = zeus::carve_workspace(ws_base, pb->n_starts, pb->dim);
  L.stream = stream;
  zeus_context::Pending pend{};
  const bool prof = ctx->profiling;
  if (prof)
    for (auto &ev : pend.ev)
      if (hipEventCreate(&ev) != hipSuccess) return fail(ZEUS_EHIP, "hipEventCreate failed");
  hipError_t e;
  if (prof) (void)hipEventRecord(pend.ev[0], stream);
  if ((e = zeus::launch_ws_init(L)) != hipSuccess) return hip_fail(e, "workspace init launch");
  if ((e = zeus::launch_pso_init(L)) != hipSuccess) return hip_fail(e, "swarm init launch");
  for (int t = 1; t <= pb->iter_pso; ++t)
    if ((e = zeus::launch_pso_step(L, t)) != hipSuccess) return hip_fail(e, "swarm update launch");
  if ((e = zeus::launch_pso_finish(L)) != hipSuccess) return hip_fail(e, "swarm best launch");
  if (prof) (void)hipEventRecord(pend.ev[1], stream);
  if ((e = zeus::launch_bfgs(L)) != hipSuccess) return hip_fail(e, "BFGS launch");
  if (prof) (void)hipEventRecord(pend.ev[2], stream);
  if ((e = zeus::launch_summary(L)) != hipSuccess) return hip_fail(e, "summary launch");
  if (prof) (void)hipEventRecord(pend.ev[3], stream);
  const size_t nd = sizeof(double) * (size_t)pb->n_starts * pb->dim;
  const size_t n8 = sizeof(double) * (size_t)pb->n_starts;
  struct Copy {
    void *dst;
    const void *src;
    size_t bytes;
  } copies[] = {{out->seeds, L.ws.x, nd}, {out->pso_v, L.ws.v, nd}, {out->pso_px, L.ws.px, nd},
                {out->pso_pf, L.ws.pf, n8}, {out->pso_best_x, L.ws.gx, sizeof(double) * pb->dim}};
  for (auto &c : copies)
    if (c.dst && (e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
      return hip_fail(e, "hipMemcpyAsync");
  if (prof) {
    ctx->pending.push_back(pend);
    ctx->prof.pso_launches += 3 + pb->iter_pso;
    ctx->prof.bfgs_launches += 1;
    ctx->prof.reduce_launches += 1;
  }
  return ZEUS_OK;
}

}  // namespace

extern "C" {

uint32_t zeus_abi_version(void) { return ZEUS_ABI_VERSION; }

const char *zeus_version(void) { return "zeus-mi355x 0.1.0 (gfx950)"; }

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
  *bytes = zeus::workspace_bytes(problem->n_starts, problem->dim);
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
    (void)drain_profile(ctx);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->res) (void)hipFree(ctx->res);
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

zeus_err zeus_minimize_async(zeus_context *ctx, const zeus_problem *problem, void *workspace,
                             size_t workspace_bytes, const zeus_result *out, void *stream) {
  g_last_error.clear();
  if (!ctx) return fail(ZEUS_EINVAL, "ctx is NULL");
  zeus_err e = check_problem(problem);
  if (e != ZEUS_OK) return e;
  if ((e = check_result(out, problem)) != ZEUS_OK) return e;
  const zeus_problem pb = *problem;
  const size_t need = zeus::workspace_bytes(pb.n_starts, pb.dim);
  if (!workspace || workspace_bytes < need)
    return fail(ZEUS_EINVAL, "workspace missing or smaller than zeus_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(ZEUS_EINVAL, "workspace must be 256-byte aligned");
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
  return enqueue_solve(ctx, &pb, workspace, out, s);
}

zeus_err zeus_minimize(zeus_context *ctx, const zeus_problem *problem, const zeus_result *out) {
  g_last_error.clear();
  if (!ctx) return fail(ZEUS_EINVAL, "ctx is NULL");
  zeus_err e = check_problem(problem);
  if (e != ZEUS_OK) return e;
  if ((e = check_result(out, problem)) != ZEUS_OK) return e;
  const zeus_problem pb = *problem;
  const size_t n = (size_t)pb.n_starts, d = (size_t)pb.dim;
  const size_t tl = out->trace ? (size_t)out->trace_len : 0;
  // device result layout (each piece 256-aligned)
  size_t off_f = 0, off_x, off_it, off_st, off_ls, off_seed, off_v, off_px, off_pf, off_gx,
         off_tr, off_sum, total;
  {
    size_t o = 0;
    off_f = o; o += align_up(8 * n);
    off_x = o; o += align_up(8 * n * d);
    off_it = o; o += align_up(4 * n);
    off_st = o; o += align_up(4 * n);
    off_ls = o; o += out->ls_trials ? align_up(4 * n) : 0;
    off_seed = o; o += out->seeds ? align_up(8 * n * d) : 0;
    off_v = o; o += out->pso_v ? align_up(8 * n * d) : 0;
    off_px = o; o += out->pso_px ? align_up(8 * n * d) : 0;
    off_pf = o; o += out->pso_pf ? align_up(8 * n) : 0;
    off_gx = o; o += out->pso_best_x ? align_up(8 * d) : 0;
    off_tr = o; o += tl ? align_up(8 * n * tl * d) : 0;
    off_sum = o; o += align_up(sizeof(zeus_summary));
    total = o;
  }
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if ((e = ensure(&ctx->ws, &ctx->ws_cap, zeus::workspace_bytes(pb.n_starts, pb.dim))) != ZEUS_OK)
    return e;
  if ((e = ensure(&ctx->res, &ctx->res_cap, total)) != ZEUS_OK) return e;
  char *R = static_cast<char *>(ctx->res);
  zeus_result dev{};
  dev.f = reinterpret_cast<double *>(R + off_f);
  dev.x = reinterpret_cast<double *>(R + off_x);
  dev.iters = reinterpret_cast<int32_t *>(R + off_it);
  dev.status = reinterpret_cast<int32_t *>(R + off_st);
  dev.ls_trials = out->ls_trials ? reinterpret_cast<int32_t *>(R + off_ls) : nullptr;
  dev.seeds = out->seeds ? reinterpret_cast<double *>(R + off_seed) : nullptr;
  dev.pso_v = out->pso_v ? reinterpret_cast<double *>(R + off_v) : nullptr;
  dev.pso_px = out->pso_px ? reinterpret_cast<double *>(R + off_px) : nullptr;
  dev.pso_pf = out->pso_pf ? reinterpret_cast<double *>(R + off_pf) : nullptr;
  dev.pso_best_x = out->pso_best_x ? reinterpret_cast<double *>(R + off_gx) : nullptr;
  dev.trace = tl ? reinterpret_cast<double *>(R + off_tr) : nullptr;
  dev.trace_len = (int32_t)tl;
  dev.summary = reinterpret_cast<zeus_summary *>(R + off_sum);
  if ((e = enqueue_solve(ctx, &pb, ctx->ws, &dev, ctx->stream)) != ZEUS_OK) return e;
  hipError_t he;
  struct Back {
    void *dst;
    const void *src;
    size_t bytes;
  } backs[] = {{out->f, dev.f, 8 * n},
               {out->x, dev.x, 8 * n * d},
               {out->iters, dev.iters, 4 * n},
               {out->status, dev.status, 4 * n},
               {out->ls_trials, dev.ls_trials, 4 * n},
               {out->seeds, dev.seeds, 8 * n * d},
               {out->pso_v, dev.pso_v, 8 * n * d},
               {out->pso_px, dev.pso_px, 8 * n * d},
               {out->pso_pf, dev.pso_pf, 8 * n},
               {out->pso_best_x, dev.pso_best_x, 8 * d},
               {out->trace, dev.trace, 8 * n * tl * d},
               {out->summary, dev.summary, sizeof(zeus_summary)}};
  for (auto &b : backs)
    if (b.dst && b.bytes &&
        (he = hipMemcpyAsync(b.dst, b.src, b.bytes, hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess)
      return hip_fail(he, "hipMemcpyAsync D2H");
  if ((he = hipStreamSynchronize(ctx->stream)) != hipSuccess)
    return hip_fail(he, "hipStreamSynchronize");
  return ZEUS_OK;
}

}  // extern "C"
