// zeus_server.cpp -- the serving loop of include/zeus.h (zeus_server_*):
// continuous batching at the level of starts.
//
//  * Requests queue in arrival order.  The oldest is admitted as soon as its
//    own device memory (result arrays, swarm state, early-stop state and a
//    one-request table) fits in the free part of the budget, and that memory
//    returns to the budget the moment its results have reached the caller.
//    Nothing but memory limits the requests in flight.
//  * An admitted request runs its swarm (Alg. 2 / 3) on the swarm stream.
//  * BFGS runs in steps.  A step is one persistent BFGS launch over slices of
//    the starts of the swarm-finished requests of one kernel class
//    (objective, precision, method, lanes); every such request gets an equal
//    share of the step, so a short request is not queued behind a long one.
//    Inside a step a group of lanes takes the next start of any slice when
//    its start retires (the slices form the launch's request table, each
//    entry naming its first start).  A step runs about four starts per
//    resident group, and two steps run at a time on two streams, so a step's
//    tail overlaps the next step and a new request joins within a step.
//  * A request with early stop runs whole in a step of its own: its stop
//    depends on all its starts (two passes on the device, no host round
//    trip).
//  * When all starts of a request have run, its best-of-N (Alg. 7) and the
//    copies into the caller's arrays run on the finish stream.
// One scheduling thread makes every device call; it polls HIP events while
// work is in flight and sleeps otherwise.  The same scheduler drives an
// emulated device (zeus_server_create_emulated) whose operations take
// modelled host time, so that admission, queueing and cancellation can be
// tested without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "zeus_host.h"
#include "zeus_internal.h"

using namespace zeus::host;

namespace {

enum State { kQueued, kSwarm, kReady, kFinishing, kDone, kCancelled, kFailed };

// An operation in flight: an event recorded after it on the device, or the
// host time at which it ends on the emulated device.
struct Op {
  hipEvent_t ev = nullptr;
  uint64_t due_ns = 0;
};

// The kernel class of a request: the slices of one step share it.
struct Klass {
  int objective, precision, method, lanes;
  bool operator<(const Klass &o) const {
    return std::tie(objective, precision, method, lanes) <
           std::tie(o.objective, o.precision, o.method, o.lanes);
  }
  bool operator==(const Klass &o) const { return !(*this < o) && !(o < *this); }
};

struct Req {
  uint64_t id = 0;
  zeus_problem pb{};
  zeus_result out{};       // the caller's host arrays
  State state = kQueued;
  zeus_err err = ZEUS_OK;
  std::string msg;
  zeus_request_times times{};
  Klass klass{};
  bool whole = false;      // early stop: one step of its own
  size_t bytes = 0, off = 0;
  // device pieces, from admission
  ResLayout rl{};
  zeus_result dev{};
  zeus::Workspace ws{};
  GroupRun own;            // its one-request group (swarm, summary)
  int64_t next = 0;        // first start not yet given to a step
  int64_t done = 0;        // starts of finished steps
  int inflight = 0;        // slices in running steps
  Op op;                   // its swarm, then its finish
};

struct Slice {
  Req *req;
  int64_t first, count;
};

struct Step {
  Klass klass{};
  std::vector<Slice> slices;
  int64_t starts = 0;
  GroupRun run;
  Op op;
};

// Most slices (table entries) of a step (fewer if its buffer is small), and
// the smallest slice a request gets while it has that many starts left.
constexpr int kMaxSlices = 1024;
constexpr int64_t kMinSlice = 256;
// Steps in flight, each with a buffer of the step arena: its header and
// table, then (wide problems) its H slots.
constexpr int kSteps = 2;
size_t step_table_bytes(size_t slices) { return kHdrBytes + table_bytes((int)slices); }

// Device bytes of a request's own block: results, workspace, its one-request
// header and table.
size_t request_bytes(const zeus_problem &pb, const zeus_result &out) {
  return align_up(res_layout(pb, out).total) + align_up(request_ws_bytes(pb)) + kHdrBytes +
         table_bytes(1);
}

// Bytes of one H slot of a wide problem of dimension d.
size_t hslot_one(int d) { return sizeof(double) * (size_t)d * (size_t)zeus::wide_cs(d); }

class Device {
 public:
  virtual ~Device() = default;
  virtual zeus_err init(size_t budget) = 0;  // allocates the budget, creates streams
  virtual char *base() = 0;
  virtual void thread_init() {}
  virtual zeus_err swarm(Req &r, char *block) = 0;
  // a step in buffer b (of kSteps) of the step arena
  virtual zeus_err step(Step &s, int b, char *buf, size_t bytes) = 0;
  virtual zeus_err finish(Req &r) = 0;
  // 1: the operation has ended, 0: still running, -1: it failed (*msg)
  virtual int poll(Op &op, std::string *msg) = 0;
  virtual int64_t resident(const Klass &k) = 0;  // starts one BFGS launch runs at once
  virtual void drain() = 0;                     // waits for everything enqueued
  virtual void release() = 0;                   // frees the budget and streams
};

// ---------------------------------------------------------------------------
// The GPU.
// ---------------------------------------------------------------------------
class HipDevice : public Device {
 public:
  explicit HipDevice(int device) : device_(device) {}

  zeus_err init(size_t budget) override {
    DeviceGuard g(device_);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = hipMalloc(&mem_, budget);
    if (e != hipSuccess) {
      mem_ = nullptr;
      return fail(ZEUS_ENOMEM, std::string("hipMalloc of the budget: ") + hipGetErrorString(e));
    }
    for (auto &st : streams_)
      if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) {
        release();
        return hip_fail(e, "hipStreamCreate");
      }
    return ZEUS_OK;
  }
  char *base() override { return static_cast<char *>(mem_); }
  void thread_init() override { (void)hipSetDevice(device_); }

  // Table upload, counter reset, swarm sweeps, swarm best and the optional
  // swarm-state copies of one admitted request, on the swarm stream.
  zeus_err swarm(Req &r, char *block) override {
    TraceRange tr("zeus.server.swarm");
    hipStream_t s = streams_[kSwarmStream];
    char *res = block, *ws = block + align_up(r.rl.total);
    char *tab = ws + align_up(request_ws_bytes(r.pb));
    r.dev = carve_result(res, r.rl, r.out);
    r.ws = carve_request_ws(ws, r.pb);
    std::vector<Planned> one{Planned{&r.pb, r.dev, r.ws}};
    zeus_err e = build_group(one, tab, nullptr, s, &r.own, false);
    if (e == ZEUS_OK) e = upload_group(r.own, s);
    if (e != ZEUS_OK) return e;
    const zeus::Group &g = r.own.g;
    hipError_t he = zeus::launch_ws_init(g);
    for (int t = 0; he == hipSuccess && t <= g.max_iter_pso; ++t) he = zeus::launch_pso(g, t);
    if (he == hipSuccess) he = zeus::launch_pso_finish(g);
    if (he != hipSuccess) return hip_fail(he, "swarm launch");
    if ((e = enqueue_copies(one, s)) != ZEUS_OK) return e;
    return record(r.op, s);
  }

  // One BFGS launch over the step's slices (two passes for a request with
  // early stop) on the stream of its buffer.
  zeus_err step(Step &st, int b, char *buf, size_t bytes) override {
    TraceRange tr("zeus.server.step");
    hipStream_t s = streams_[b == 0 ? kStepStream0 : kStepStream1];
    std::vector<zeus_problem> pbs(st.slices.size());
    std::vector<Planned> planned(st.slices.size());
    for (size_t k = 0; k < st.slices.size(); ++k) {
      const Slice &sl = st.slices[k];
      pbs[k] = sl.req->pb;
      pbs[k].n_starts = sl.count;
      planned[k] = Planned{&pbs[k], sl.req->dev, sl.req->ws};
    }
    char *hs = buf + step_table_bytes(st.slices.size());
    const size_t hs_bytes = bytes - step_table_bytes(st.slices.size());
    zeus_err e = build_group(planned, buf, hs, s, &st.run);
    if (e != ZEUS_OK) return e;
    for (size_t k = 0; k < st.slices.size(); ++k) st.run.host[k].slice_first = st.slices[k].first;
    zeus::Group &g = st.run.g;
    if (g.method == 0 && g.g_bfgs == zeus::kWideLanes) {
      // as many H slots (one per resident block) as the buffer holds
      const int64_t fit = (int64_t)(hs_bytes / hslot_one(max_dim(planned)));
      if (fit < 1) return fail(ZEUS_ENOMEM, "step buffer holds no H slot");
      if (g.wide_slots > fit) g.wide_slots = (int)fit;
    }
    if ((e = upload_group(st.run, s)) != ZEUS_OK) return e;
    hipError_t he = zeus::launch_ws_init(g);
    if (he == hipSuccess) he = zeus::launch_bfgs(g);
    if (he == hipSuccess && g.early_stop) {
      he = zeus::launch_es_finish(g);
      if (he == hipSuccess) he = zeus::launch_bfgs(g);
    }
    if (he != hipSuccess) return hip_fail(he, "BFGS launch");
    return record(st.op, s);
  }

  // Best-of-N and the copies into the caller's arrays, on the finish stream.
  zeus_err finish(Req &r) override {
    TraceRange tr("zeus.server.finish");
    hipStream_t s = streams_[kFinishStream];
    zeus::Group g = r.own.g;
    g.stream = s;
    hipError_t he = zeus::launch_summary(g);
    if (he != hipSuccess) return hip_fail(he, "summary launch");
    zeus_err e = copy_back(r.pb, r.out, r.dev, s);
    if (e != ZEUS_OK) return e;
    return record(r.op, s);
  }

  int poll(Op &op, std::string *msg) override {
    if (!op.ev) return 1;
    const hipError_t e = hipEventQuery(op.ev);
    if (e == hipErrorNotReady) return 0;
    (void)hipEventDestroy(op.ev);
    op.ev = nullptr;
    if (e == hipSuccess) return 1;
    *msg = std::string("device error: ") + hipGetErrorString(e);
    return -1;
  }

  int64_t resident(const Klass &k) override {
    zeus::Group g{};
    g.objective = k.objective;
    g.precision = k.precision;
    g.method = k.method;
    g.g_bfgs = k.lanes;
    g.total_starts = 1;
    g.wide_slots = zeus::kWideMaxSlots;
    int64_t out = 0;
    g.resident = &out;
    if (zeus::launch_bfgs(g) != hipSuccess || out < 1) out = 1024;
    return out;
  }

  void drain() override {
    for (auto &st : streams_)
      if (st) (void)hipStreamSynchronize(st);
  }

  void release() override {
    DeviceGuard g(device_);
    drain();
    for (auto &st : streams_)
      if (st) {
        (void)hipStreamDestroy(st);
        st = nullptr;
      }
    if (mem_) (void)hipFree(mem_);
    mem_ = nullptr;
  }

 private:
  zeus_err record(Op &op, hipStream_t s) {
    hipError_t e = hipEventCreateWithFlags(&op.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(op.ev, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return ZEUS_OK;
  }

  // Four streams (the hardware queues a process gets by default): the swarm,
  // one per step buffer, and the finish.
  enum { kSwarmStream, kStepStream0, kStepStream1, kFinishStream, kStreams };
  int device_;
  void *mem_ = nullptr;
  hipStream_t streams_[kStreams] = {};
};
static_assert(kSteps == 2, "one stream per step buffer");

// ---------------------------------------------------------------------------
// The emulated device: modelled host time, placeholder results.
// ---------------------------------------------------------------------------
class EmulatedDevice : public Device {
 public:
  explicit EmulatedDevice(const zeus_emulation &e) : emu_(e) {}
  zeus_err init(size_t) override { return ZEUS_OK; }
  // Addresses are only ever computed, never dereferenced.
  char *base() override { return reinterpret_cast<char *>(uintptr_t(1) << 44); }
  zeus_err swarm(Req &r, char *) override {
    r.op.due_ns = now_ns() + emu_.swarm_ns;
    return ZEUS_OK;
  }
  zeus_err step(Step &s, int, char *, size_t) override {
    const int64_t rounds = (s.starts + emu_.resident_starts - 1) / emu_.resident_starts;
    s.op.due_ns = now_ns() + emu_.step_ns + (uint64_t)rounds * emu_.start_ns;
    return ZEUS_OK;
  }
  zeus_err finish(Req &r) override {
    const size_t n = (size_t)r.pb.n_starts, d = (size_t)r.pb.dim;
    for (size_t i = 0; i < n; ++i) {
      r.out.f[i] = (double)r.pb.request_id;
      r.out.iters[i] = 0;
      r.out.status[i] = ZEUS_ST_MAXITER;
      if (r.out.ls_trials) r.out.ls_trials[i] = 0;
      if (r.out.skips) r.out.skips[i] = 0;
      if (r.out.resets) r.out.resets[i] = 0;
    }
    std::memset(r.out.x, 0, sizeof(double) * n * d);
    zeus_summary s{};
    s.best_index = 0;
    s.best_f = (double)r.pb.request_id;
    s.pso_best_f = (double)r.pb.request_id;
    *r.out.summary = s;
    r.op.due_ns = now_ns() + emu_.finish_ns;
    return ZEUS_OK;
  }
  int poll(Op &op, std::string *) override { return now_ns() >= op.due_ns ? 1 : 0; }
  int64_t resident(const Klass &) override { return emu_.resident_starts; }
  void drain() override {}
  void release() override {}

 private:
  zeus_emulation emu_;
};

}  // namespace

struct zeus_server {
  std::unique_ptr<Device> dev;
  size_t budget = 0;       // bytes for requests (the pool)
  size_t step_bytes = 0;   // bytes of each step buffer
  int max_slices = 1;      // slices a step buffer's table holds
  char *pool_base = nullptr, *arena = nullptr;
  Pool pool;
  std::mutex mu;
  std::condition_variable cv;       // the scheduler: submissions, cancellations, shutdown
  std::condition_variable done_cv;  // waiters: a request ended
  std::deque<uint64_t> queue;       // queued requests in arrival order
  std::list<Req *> active;          // admitted requests in admission order
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::unique_ptr<Step> steps[kSteps];
  std::map<Klass, int64_t> resident;  // per class, from the device
  Klass last_klass{-1, -1, -1, -1};
  uint64_t next_id = 1;
  bool stopping = false;
  std::thread sched;

  void loop() {
    dev->thread_init();
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      const bool a = reap(), b = admit(), c = schedule();
      if (stopping && queue.empty() && active.empty()) break;
      if (a || b || c) continue;
      if (active.empty())
        cv.wait(lk);
      else
        cv.wait_for(lk, std::chrono::microseconds(50));
    }
  }

  // Marks a request failed; it ends once none of its work is in flight.
  void fail_req(Req &r, zeus_err e, const std::string &msg) {
    if (r.err == ZEUS_OK) {
      r.err = e;
      r.msg = msg;
    }
  }

  void end_req(Req &r, State st) {
    trace_mark("zeus.server.retire");
    r.state = st;
    r.times.t_done_ns = now_ns();
    pool.release(r.off, r.bytes);
    active.remove(&r);
    done_cv.notify_all();
  }

  bool reap() {
    bool any = false;
    std::string msg;
    for (auto &sp : steps) {
      if (!sp) continue;
      const int r = dev->poll(sp->op, &msg);
      if (r == 0) continue;
      for (const Slice &sl : sp->slices) {
        sl.req->done += sl.count;
        --sl.req->inflight;
        if (r < 0) fail_req(*sl.req, ZEUS_EHIP, msg);
      }
      sp.reset();
      any = true;
    }
    for (auto it = active.begin(); it != active.end();) {
      Req &q = **it;
      ++it;  // q may leave the list below
      if (q.state == kSwarm) {
        const int r = dev->poll(q.op, &msg);
        if (r == 0) continue;
        if (r < 0) fail_req(q, ZEUS_EHIP, msg);
        q.state = kReady;
        any = true;
      }
      if (q.state == kReady && q.inflight == 0 && (q.err != ZEUS_OK || q.done == q.pb.n_starts)) {
        any = true;
        if (q.err != ZEUS_OK) {
          end_req(q, kFailed);
          continue;
        }
        const zeus_err e = dev->finish(q);
        if (e != ZEUS_OK) {
          dev->drain();
          fail_req(q, e, g_last_error);
          end_req(q, kFailed);
          continue;
        }
        q.state = kFinishing;
      }
      if (q.state == kFinishing) {
        const int r = dev->poll(q.op, &msg);
        if (r == 0) continue;
        if (r < 0) fail_req(q, ZEUS_EHIP, msg);
        end_req(q, q.err == ZEUS_OK ? kDone : kFailed);
        any = true;
      }
    }
    return any;
  }

  // Admits queued requests, oldest first, while the oldest fits.
  bool admit() {
    bool any = false;
    while (!queue.empty()) {
      Req &q = *reqs.at(queue.front());
      size_t off = 0;
      if (!pool.alloc(q.bytes, &off)) break;
      queue.pop_front();
      trace_mark("zeus.server.admit");
      q.off = off;
      q.state = kSwarm;
      q.times.t_admit_ns = now_ns();
      active.push_back(&q);
      any = true;
      const zeus_err e = dev->swarm(q, pool_base + off);
      if (e != ZEUS_OK) {
        dev->drain();
        fail_req(q, e, g_last_error);
        q.state = kReady;  // nothing in flight: ends at the next reap
      }
    }
    return any;
  }

  // Requests of a class that can take a slice now, in admission order.
  std::vector<Req *> candidates(const Klass &k) {
    std::vector<Req *> c;
    for (Req *q : active)
      if (q->state == kReady && q->err == ZEUS_OK && q->klass == k && q->next < q->pb.n_starts)
        c.push_back(q);
    return c;
  }

  std::unique_ptr<Step> build_step() {
    // the classes with work, taken in turn after the last one served
    std::vector<Klass> ks;
    for (Req *q : active)
      if (q->state == kReady && q->err == ZEUS_OK && q->next < q->pb.n_starts &&
          std::find(ks.begin(), ks.end(), q->klass) == ks.end())
        ks.push_back(q->klass);
    if (ks.empty()) return nullptr;
    std::sort(ks.begin(), ks.end());
    auto pick = std::upper_bound(ks.begin(), ks.end(), last_klass);
    const Klass k = pick == ks.end() ? ks.front() : *pick;
    last_klass = k;
    std::vector<Req *> c = candidates(k);
    auto st = std::make_unique<Step>();
    st->klass = k;
    if (c.front()->whole) {  // early stop: the whole request alone
      Req *q = c.front();
      st->slices.push_back(Slice{q, 0, q->pb.n_starts});
      st->starts = q->pb.n_starts;
      q->next = q->pb.n_starts;
      ++q->inflight;
      return st;
    }
    auto res = resident.find(k);
    if (res == resident.end()) res = resident.emplace(k, dev->resident(k)).first;
    const int64_t target = 4 * res->second;
    int64_t parts = 0;
    for (Req *q : c) parts += q->whole ? 0 : 1;
    const int64_t quota = std::max<int64_t>(kMinSlice, (target + parts - 1) / parts);
    for (Req *q : c) {
      if (q->whole) continue;
      const int64_t take = std::min<int64_t>(quota, q->pb.n_starts - q->next);
      st->slices.push_back(Slice{q, q->next, take});
      st->starts += take;
      q->next += take;
      ++q->inflight;
      if (st->starts >= target || (int)st->slices.size() == max_slices) break;
    }
    return st;
  }

  bool schedule() {
    bool any = false;
    for (int b = 0; b < kSteps; ++b) {
      if (steps[b]) continue;
      std::unique_ptr<Step> st = build_step();
      if (!st) break;
      any = true;
      const zeus_err e = dev->step(*st, b, arena + (size_t)b * step_bytes, step_bytes);
      if (e != ZEUS_OK) {
        dev->drain();
        const std::string msg = g_last_error;
        for (const Slice &sl : st->slices) {
          --sl.req->inflight;
          fail_req(*sl.req, e, msg);
        }
        continue;
      }
      steps[b] = std::move(st);
    }
    return any;
  }
};

namespace {

// Creates a server over `dev`: a quarter of the budget (at most 2 GiB) for
// the step buffers, the rest for requests.
zeus_err create_server(std::unique_ptr<Device> dev, size_t hbm_budget_bytes, zeus_server **out) {
  if (hbm_budget_bytes < ((size_t)1 << 20)) return fail(ZEUS_EINVAL, "budget below 1 MiB");
  auto srv = std::unique_ptr<zeus_server>(new (std::nothrow) zeus_server);
  if (!srv) return fail(ZEUS_ENOMEM, "server allocation failed");
  const size_t total = hbm_budget_bytes / kAlign * kAlign;
  const size_t arena = std::min<size_t>(total / 4, (size_t)2 << 30) / (kAlign * kSteps) * (kAlign * kSteps);
  srv->step_bytes = arena / kSteps;
  if (srv->step_bytes < step_table_bytes(1)) return fail(ZEUS_EINVAL, "budget too small for a step");
  srv->max_slices =
      (int)std::min<size_t>(kMaxSlices, (srv->step_bytes - kHdrBytes) / sizeof(zeus::ReqDev));
  srv->budget = total - arena;
  zeus_err e = dev->init(total);
  if (e != ZEUS_OK) return e;
  srv->dev = std::move(dev);
  srv->arena = srv->dev->base();
  srv->pool_base = srv->arena + arena;
  srv->pool.reset(srv->budget);
  zeus_server *raw = srv.get();
  raw->sched = std::thread([raw] { raw->loop(); });
  *out = srv.release();
  return ZEUS_OK;
}

}  // namespace

extern "C" {

zeus_err zeus_server_create(zeus_context *ctx, size_t hbm_budget_bytes, zeus_server **out) {
  g_last_error.clear();
  if (!ctx || !out) return fail(ZEUS_EINVAL, "NULL argument");
  *out = nullptr;
  return create_server(std::unique_ptr<Device>(new HipDevice(context_device(ctx))),
                       hbm_budget_bytes, out);
}

zeus_err zeus_server_create_emulated(size_t hbm_budget_bytes, const zeus_emulation *emu,
                                     zeus_server **out) {
  g_last_error.clear();
  if (!emu || !out) return fail(ZEUS_EINVAL, "NULL argument");
  *out = nullptr;
  if (emu->resident_starts < 1) return fail(ZEUS_EINVAL, "resident_starts must be >= 1");
  return create_server(std::unique_ptr<Device>(new EmulatedDevice(*emu)), hbm_budget_bytes, out);
}

zeus_err zeus_server_request_bytes(const zeus_problem *problem, const zeus_result *host_out,
                                   size_t *bytes) {
  g_last_error.clear();
  if (!bytes) return fail(ZEUS_EINVAL, "bytes is NULL");
  zeus_err e = check_problem(problem);
  if (e == ZEUS_OK) e = check_result(host_out, problem);
  if (e != ZEUS_OK) return e;
  zeus_result out = *host_out;
  if (!out.trace || out.trace_len == 0) {
    out.trace = nullptr;
    out.trace_len = 0;
  }
  *bytes = request_bytes(*problem, out);
  return ZEUS_OK;
}

zeus_err zeus_server_submit(zeus_server *srv, const zeus_problem *problem,
                            const zeus_result *host_out, uint64_t *ticket) {
  g_last_error.clear();
  if (!srv || !ticket) return fail(ZEUS_EINVAL, "NULL argument");
  zeus_err e = check_problem(problem);
  if (e == ZEUS_OK) e = check_result(host_out, problem);
  if (e != ZEUS_OK) return e;
  auto r = std::make_unique<Req>();
  r->pb = *problem;
  r->out = *host_out;
  if (!r->out.trace || r->out.trace_len == 0) {
    r->out.trace = nullptr;
    r->out.trace_len = 0;
  }
  r->klass = Klass{r->pb.objective, r->pb.precision, method_of(r->pb), lanes_of(r->pb)};
  r->whole = r->pb.required_converged > 0;
  r->rl = res_layout(r->pb, r->out);
  r->bytes = request_bytes(r->pb, r->out);
  if (r->bytes > srv->budget)
    return fail(ZEUS_ENOMEM, "request needs " + std::to_string(r->bytes) +
                                 " bytes of device memory, more than the server's budget for "
                                 "requests (" + std::to_string(srv->budget) + ")");
  if (hslot_lanes(r->pb) == zeus::kWideLanes &&
      srv->step_bytes < step_table_bytes(1) + hslot_one(r->pb.dim))
    return fail(ZEUS_ENOMEM, "budget too small for one inverse-Hessian slot of this dimension");
  r->times.t_submit_ns = now_ns();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stopping) return fail(ZEUS_ECANCELLED, "server is shutting down");
  const uint64_t id = srv->next_id++;
  r->id = id;
  srv->queue.push_back(id);
  srv->reqs.emplace(id, std::move(r));
  *ticket = id;
  srv->cv.notify_one();
  return ZEUS_OK;
}

zeus_err zeus_server_wait(zeus_server *srv, uint64_t ticket, int64_t timeout_ns,
                          zeus_request_times *times) {
  g_last_error.clear();
  if (!srv) return fail(ZEUS_EINVAL, "srv is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  const auto deadline =
      std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns > 0 ? timeout_ns : 0);
  for (;;) {
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(ZEUS_EINVAL, "unknown or released ticket");
    Req &r = *it->second;
    if (r.state == kDone || r.state == kCancelled || r.state == kFailed) {
      if (times) *times = r.times;
      const State st = r.state;
      const zeus_err err = r.err;
      const std::string msg = r.msg;
      srv->reqs.erase(it);
      if (st == kDone) return ZEUS_OK;
      if (st == kCancelled) return fail(ZEUS_ECANCELLED, "request was cancelled");
      return fail(err, msg);
    }
    if (timeout_ns == 0) return ZEUS_NOT_READY;
    if (timeout_ns < 0) {
      srv->done_cv.wait(lk);
    } else if (srv->done_cv.wait_until(lk, deadline) == std::cv_status::timeout) {
      auto again = srv->reqs.find(ticket);
      if (again != srv->reqs.end() && again->second->state != kDone &&
          again->second->state != kCancelled && again->second->state != kFailed)
        return fail(ZEUS_ETIMEOUT, "timed out");
    }
  }
}

zeus_err zeus_server_cancel(zeus_server *srv, uint64_t ticket) {
  g_last_error.clear();
  if (!srv) return fail(ZEUS_EINVAL, "srv is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return fail(ZEUS_EINVAL, "unknown or released ticket");
  Req &r = *it->second;
  if (r.state != kQueued) {
    if (r.state == kDone || r.state == kCancelled || r.state == kFailed) return ZEUS_OK;
    g_last_error = "request is running; wait for it";
    return ZEUS_NOT_READY;
  }
  srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), ticket));
  r.state = kCancelled;
  r.times.t_done_ns = now_ns();
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
    for (uint64_t id : srv->queue) {
      srv->reqs.at(id)->state = kCancelled;
      srv->reqs.at(id)->times.t_done_ns = now_ns();
    }
    srv->queue.clear();
    srv->cv.notify_all();
    srv->done_cv.notify_all();
  }
  srv->sched.join();  // the admitted requests end first
  srv->dev->release();
  delete srv;
  return ZEUS_OK;
}

}  // extern "C"
