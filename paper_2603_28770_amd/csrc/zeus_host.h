// zeus_host.h -- host-side pieces shared by the C-ABI translation units
// (zeus_api.cpp: validation, planning, launch sequences and the blocking,
// asynchronous and captured entry points; zeus_server.cpp: the serving
// loop).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "zeus_internal.h"

struct zeus_context;

namespace zeus {
namespace host {

// The calling thread's last error message (zeus_last_error).
extern thread_local std::string g_last_error;

zeus_err fail(zeus_err e, const std::string &msg);
zeus_err hip_fail(hipError_t e, const char *what);

// roctx ranges and markers on the host timeline (rocprofv3 --marker-trace):
// a range around each entry point and each launch phase, markers where the
// server admits and retires a request.  Without a profiler attached they
// cost a call each.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};
inline void trace_mark(const char *what) { roctxMarkA(what); }

// Device memory pieces are 256-byte aligned.
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Argument checks shared by every entry point taking a problem (user: a
// ZEUS_USER problem of zeus_minimize_user).
zeus_err check_problem(const zeus_problem *p, bool user = false);
zeus_err check_result(const zeus_result *r, const zeus_problem *p);

// Makes `dev` current for the guard's lifetime.
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

// A launch group's header (BatchDev, padded) precedes its request table.
constexpr size_t kHdrBytes = 256;
inline size_t table_bytes(int nreq) { return align_up(sizeof(ReqDev) * (size_t)nreq); }

// One request of a launch group: its problem, device outputs and workspace.
struct Planned {
  const zeus_problem *pb;
  zeus_result dev;  // device pointers
  Workspace ws;
};

int max_dim(const std::vector<Planned> &reqs);
// Device bytes of the H slots a group needs (0 unless its problems are wide).
size_t hslot_bytes(int g_bfgs, int64_t total_starts, int dmax);
// Method (0 BFGS, 1 L-BFGS) and lanes / coordinate slots per start.
int method_of(const zeus_problem &p);
int lanes_of(const zeus_problem &p);
// Lanes whose BFGS kernel keeps H in device-memory slots (0 for L-BFGS).
int hslot_lanes(const zeus_problem &p);
// A request's device workspace: swarm state and early-stop state.
size_t request_ws_bytes(const zeus_problem &p);
Workspace carve_request_ws(void *base, const zeus_problem &p);

// A launch group ready to run: the kernels' view (Group) and the host copy of
// its request table.
struct GroupRun {
  Group g;
  std::vector<ReqDev> host;
};

// Builds the launch group of requests that share objective, precision and
// lane counts (nothing is enqueued); hdr_table is the group's header
// followed by its table, hslots its H slots (wide problems only; a group that
// will not run BFGS may go without, need_hslots false).
zeus_err build_group(const std::vector<Planned> &reqs, void *hdr_table, void *hslots,
                     hipStream_t stream, GroupRun *run, bool need_hslots = true);
zeus_err upload_group(const GroupRun &run, hipStream_t stream);
// Device copies of the optional swarm-state outputs.
zeus_err enqueue_copies(const std::vector<Planned> &reqs, hipStream_t stream);
// Enqueues a group's kernels on its stream: counter reset, (with_swarm) the
// swarm sweeps and best, BFGS (two passes with early stop), one summary per
// request, then (with_copies) the swarm-state copies.  ctx may be null
// (no profiling, no user objective).
zeus_err launch_group(zeus_context *ctx, const GroupRun &run, const std::vector<Planned> &reqs,
                      bool with_copies, bool with_swarm = true);
// Build, upload and launch one group on `stream`.
zeus_err enqueue_group(zeus_context *ctx, const std::vector<Planned> &reqs, void *hdr_table,
                       void *hslots, hipStream_t stream);

// Device result arrays of one request laid out in one piece of memory (the
// optional outputs only where the caller asked for them).
struct ResLayout {
  size_t f, x, it, st, ls, sk, rs, seed, v, px, pf, gx, tr, sum, total;
};
ResLayout res_layout(const zeus_problem &pb, const zeus_result &out);
zeus_result carve_result(char *R, const ResLayout &l, const zeus_result &out);
// Copies the device results into the caller's host arrays (on stream s).
zeus_err copy_back(const zeus_problem &pb, const zeus_result &out, const zeus_result &dev,
                   hipStream_t s);

// Host steady clock in nanoseconds.
uint64_t now_ns();

// The device of a context.
int context_device(const zeus_context *ctx);

// First-fit allocator over [0, size) of one device allocation.
class Pool {
 public:
  void reset(size_t size);
  bool alloc(size_t bytes, size_t *off);
  void release(size_t off, size_t bytes);
  size_t largest() const;
  size_t free_bytes() const;

 private:
  std::map<size_t, size_t> free_;  // offset -> size
};

}  // namespace host
}  // namespace zeus
