// zeus_pso.hip -- swarm phase on gfx950: the kernel launches (the kernel
// templates are in zeus_pso_kernels.h), the swarm-best publication and the
// per-launch work-counter reset.
#include "zeus_pso_kernels.h"

namespace zeus {
namespace {

// Stage (3): publish every request's swarm best after its last sweep (one
// block per request).
__global__ __launch_bounds__(kPsoBlock) void pso_finish_kernel(const ReqDev *reqs) {
  __shared__ double gx_sh[kMaxDim];
  const ReqDev &a = reqs[blockIdx.x];
  StageTwo<kPsoBlock> s2;
  stage_two_load<kPsoBlock>(a, a.iter_pso, s2);
  global_best_after<kPsoBlock>(a, a.iter_pso, gx_sh, true, a.ws.best, a.ws.gx, s2);
}

// Before a group's launches: the BFGS work counter and the early-stop pass,
// and (block r) the early-stop state of request r when it stops early.
__global__ __launch_bounds__(256) void ws_init_kernel(BatchDev *hdr, const ReqDev *reqs,
                                                      int early_stop) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hdr->queue = 0ull;
    hdr->es_pass = early_stop ? 1u : 0u;
  }
  const ReqDev &rq = reqs[blockIdx.x];
  if (!rq.ws.es) return;
  const int len = es_ints(rq.iter_bfgs);
  for (int i = threadIdx.x; i < len; i += blockDim.x)
    rq.ws.es[i] = i == kEsBound ? rq.iter_bfgs : i == kEsKstar ? -1 : 0;
}

template <int OBJ, int G, int CPL = 1>
hipError_t launch_g(const Group &g, int t) {
  hipLaunchKernelGGL((pso_kernel<OBJ, G, CPL>), dim3(g.pso_grid), dim3(pso_threads(G * CPL)), 0, g.stream,
                     g.reqs, g.nreq, t);
  return hipGetLastError();
}

// Swarm slots (the power of two >= dim) from 8 on run as slots / 4 lanes of
// four coordinates each: a wave then holds four times the particles, which
// shares each particle's fixed costs (its block of the swarm loop, the
// personal-best test, the group sum's lane levels) four ways.  The sums are
// the same pairwise trees at any split.  Against one coordinate per lane the
// swarm phase took 0.91 of the time at d = 10, 0.75 (Ackley) and 0.80
// (Rosenbrock) at d = 50 and 0.94 at d = 128.
template <int OBJ>
hipError_t launch_obj(const Group &g, int t) {
  switch (g.g_pso) {
    case 2: return launch_g<OBJ, 2>(g, t);
    case 4: return launch_g<OBJ, 4>(g, t);
    case 8: return launch_g<OBJ, 2, 4>(g, t);
    case 16: return launch_g<OBJ, 4, 4>(g, t);
    case 32: return launch_g<OBJ, 8, 4>(g, t);
    case 64: return launch_g<OBJ, 16, 4>(g, t);
    case 128: return launch_g<OBJ, 32, 4>(g, t);
    case 256: return launch_g<OBJ, 64, 4>(g, t);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int pso_group_lanes(int dim) {
  int g = 2;
  while (g < dim) g <<= 1;
  return g;
}

int pso_blocks(int64_t n, int dim) {
  const int slots = pso_group_lanes(dim);
  const int lanes = slots < 64 ? slots : 64;
  const int64_t per_block = pso_threads(slots) / lanes;
  const int64_t want = (n + per_block - 1) / per_block;
  return (int)(want < kPsoMaxBlocks ? want : kPsoMaxBlocks);
}

hipError_t launch_ws_init(const Group &g) {
  hipLaunchKernelGGL(ws_init_kernel, dim3(g.nreq), dim3(256), 0, g.stream, g.hdr, g.reqs,
                     g.early_stop ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pso(const Group &g, int t) {
  switch (g.objective) {
    case kRosenbrock: return launch_obj<kRosenbrock>(g, t);
    case kRastrigin: return launch_obj<kRastrigin>(g, t);
    case kAckley: return launch_obj<kAckley>(g, t);
    case kStyblinskiTang: return launch_obj<kStyblinskiTang>(g, t);
    case kGoldsteinPrice: return launch_g<kGoldsteinPrice, 2>(g, t);
    case kSphere: return launch_obj<kSphere>(g, t);
    case kQuartic: return launch_obj<kQuartic>(g, t);
    case kUser: return launch_user_pso(g, t);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pso_finish(const Group &g) {
  hipLaunchKernelGGL(pso_finish_kernel, dim3(g.nreq), dim3(kPsoBlock), 0, g.stream, g.reqs);
  return hipGetLastError();
}

}  // namespace zeus
