// zeus_internal.h -- host-side declarations shared by the C-ABI layer and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/zeus.h"

namespace zeus {

// Largest dimension of this build.  Up to kMaxNarrowDim a group of at most one
// 64-lane wavefront runs a start with the inverse Hessian in its registers;
// up to kTileBlockDim a block of kWideLanes lanes (four wavefronts) runs a
// start with H in the registers of its wavefronts, a 64 x 64 quarter each;
// up to kHybridDim a block of eight wavefronts runs a start with eight 64 x 64
// tiles of H in its registers and the rest in LDS; above that a block of
// kWideLanes lanes runs a start with the rows in a device-memory slot of the
// block.  As a tiling (lanes per start, below), kTileBlockDim names the
// on-chip four-wavefront block, kHybridDim the register-and-LDS block and
// kWideLanes the device-memory one.
constexpr int kMaxDim = 256;
constexpr int kMaxNarrowDim = 64;
constexpr int kTileBlockDim = 128;
constexpr int kHybridDim = 208;
constexpr int kWideLanes = 256;
// Most H slots (resident wide blocks) a launch group uses.
constexpr int kWideMaxSlots = 2048;
// Most (s, y) pairs an L-BFGS start keeps (in registers).
constexpr int kLbfgsMaxHistory = 8;
constexpr int kPsoBlock = 256;
// Threads per swarm block (256 for every particle width: larger blocks lower
// the number of resident blocks per CU more than they add groups).
constexpr int pso_threads(int) { return kPsoBlock; }
constexpr int kBfgsBlock = 256;

// Most blocks a swarm launch gives one request (the blocks stride over its
// particles; each re-reduces the previous launch's block results, so this
// stays small).
constexpr int kPsoMaxBlocks = 1024;

// A swarm best, kept on the device.
struct PsoBest {
  double f;      // value as computed (may be NaN if every value is NaN)
  int64_t idx;   // particle index
};

// Device workspace of one request (all pieces 256-byte aligned).  The swarm
// kernels exchange their block results through double-buffered slots: sweep
// t writes slot t & 1, sweep t+1 reads it after the kernel boundary, so no
// launch needs a device-wide fence.
struct Workspace {
  PsoBest *best;           // swarm best after the last sweep
  double *gx;              // [dim] its position
  PsoBest *best_store;     // [2] swarm best after sweep t, slot t & 1
  double *gx_store;        // [2][dim]
  double *part_key;        // [2][P] each block's best rank key of sweep t
  double *part_f;          // [2][P] its value
  int64_t *part_idx;       // [2][P] its particle
  double *part_x;          // [2][P][dim] its personal-best position
  double *x, *v, *px;      // [n][dim]
  double *pf;              // [n]
  int32_t *es;             // early-stop state (below), nullptr without early stop
  int pso_blocks;          // P
};

// Early stop (required_converged = c > 0, Alg. 10), read iteration-
// synchronously: K* is the iteration at which the c-th start converges and
// every start still running at K* ends there.  The BFGS kernel runs twice.
// In the first pass a start that converges at iteration k adds itself to a
// Fenwick tree of convergence counts by iteration, and every start stops at
// iteration k >= bound, where bound is the c-th smallest convergence
// iteration among the starts counted so far.  Counts only grow, so bound
// only falls and never drops below K*.  After the pass the tree is complete
// up to K*, which gives K* exactly; the second pass reruns from their seeds,
// capped at K*, the starts that went past it.  The int32 state of a request:
//   es[kEsBound]          the stopping bound (starts at iter_bfgs)
//   es[kEsKstar]          K* after the first pass (-1: fewer than c converge)
//   es[kEsCount]          convergences counted so far
//   es[kEsTree + i]       Fenwick node i = 1 .. iter_bfgs + 1 (iteration i - 1)
constexpr int kEsBound = 0, kEsKstar = 1, kEsCount = 2, kEsTree = 3;
__host__ __device__ constexpr int es_ints(int iter_bfgs) { return kEsTree + iter_bfgs + 2; }

// Device bytes of one request's workspace (swarm state, and es_len ints of
// early-stop state when es_len > 0), and its pieces at `base`.
size_t workspace_bytes(int64_t n, int dim, int es_len = 0);
Workspace carve_workspace(void *base, int64_t n, int dim, int es_len = 0);

// One request of a launch as the kernels see it (a table in device memory).
// A launch serves requests that share objective, precision and lane counts.
struct ReqDev {
  int64_t n;                 // particles == starts
  int d, iter_pso, iter_bfgs, iter_ls, trace_len;
  int stop_status;           // status of a start that reaches iter_bfgs
  int lbfgs_m;               // L-BFGS pairs kept (0: BFGS)
  int pad0;
  double lo, hi, vh;         // box and velocity half-range
  double w, c1, c2;          // swarm coefficients
  double armijo_c, shrink, tol;
  uint64_t k0, k1;           // Philox key (seed, request id)
  Workspace ws;              // swarm state
  double *out_f, *out_x;     // results (device)
  int32_t *out_iters, *out_status, *out_ls;
  int32_t *out_skips, *out_resets;  // per-start update skips and descent resets (nullable)
  double *trace;
  zeus_summary *summary;
  int64_t start_offset;      // first start of this request in the BFGS launch
  int block_offset;          // first block of this request in a swarm launch
  int pad1;
  int64_t required_c;        // early stop at this many converged starts (0: off)
  int64_t slice_first;       // this entry runs starts slice_first, slice_first + 1, ...
                             // of its request (a slice of the request's starts)
};

// Shared counters of one launch group.
struct BatchDev {
  uint64_t queue;            // next unclaimed BFGS start over all requests
  uint32_t es_pass;          // 0: no early stop; 1, 2: first, second BFGS pass
  uint32_t pad;
};

// Kernels of a user objective, compiled at run time (zeus_user.cpp): the
// module, its swarm kernels by log2 of the coordinate slots per particle
// (2..256), its BFGS kernels by log2 of the lanes per start (4..64), its
// block BFGS kernels (H in registers up to d = 128, in registers and LDS up
// to 208) and its L-BFGS kernels by log2 of the coordinate slots per start
// (4..256) (hipModule_t and hipFunction_t handles).
struct UserKernels {
  void *module;
  void *pso[9];
  // [0]: FP64, [1]: mixed precision (FP32 evaluations)
  void *bfgs[2][7];
  void *bfgs_tile[2], *bfgs_hybrid[2];
  void *lbfgs[2][9];
};

// A launch group: device table of nreq requests plus its counters.
struct Group {
  int objective;
  int precision;
  int method;                // 0: BFGS, 1: L-BFGS
  int g_pso, g_bfgs;         // lanes per particle / per start
  int nreq;
  int max_iter_pso;
  int pso_grid;              // total swarm blocks (sum of P)
  int64_t total_starts;
  const ReqDev *reqs;        // device
  BatchDev *hdr;             // device
  hipStream_t stream;
  // wide problems (g_bfgs == kWideLanes): the blocks' H slots
  double *hslots;            // [wide_slots][wide_slot_doubles]
  int wide_slots;
  int wide_cs;               // column stride of a slot (max dim rounded up to 64)
  int64_t wide_slot_doubles; // max dim * wide_cs
  const UserKernels *user;   // objective == kUser: its compiled kernels
  bool early_stop;           // some request has required_converged > 0
  int64_t *resident;         // non-null: the BFGS launcher only stores here how many
                             // starts its kernel keeps resident at once (no launch)
};

// H slots of a wide launch group whose largest dimension is dmax.
int wide_slots(int64_t total_starts);
int wide_cs(int dmax);
size_t wide_hslot_bytes(int64_t total_starts, int dmax);

// Kernel launchers (return the first HIP error, hipSuccess otherwise).
hipError_t launch_ws_init(const Group &g);
// After the first BFGS pass of a group with early stop: K* of every such
// request, and the work counter reset for the second pass.
hipError_t launch_es_finish(const Group &g);
hipError_t launch_pso(const Group &g, int t);
hipError_t launch_pso_finish(const Group &g);
hipError_t launch_bfgs(const Group &g);
hipError_t launch_bfgs_wide(const Group &g, int cus);
hipError_t launch_bfgs_tile(const Group &g, int cus);
hipError_t launch_bfgs_hybrid(const Group &g, int cus);
hipError_t launch_lbfgs(const Group &g, int cus);
// Coordinate slots per L-BFGS start (power of two >= max(dim, 4); one
// wavefront covers up to 256).
int lbfgs_slots(int dim);
hipError_t launch_summary(const Group &g);
// User objectives: swarm sweep, (d <= 64) BFGS and L-BFGS launches of the
// compiled kernels, and the dynamic LDS of a BFGS block with `lanes` lanes per
// start and of an L-BFGS block with `slots` coordinate slots per start.
hipError_t launch_user_pso(const Group &g, int t);
hipError_t launch_user_bfgs(const Group &g, int64_t want, int cus);
hipError_t launch_user_lbfgs(const Group &g, int cus);
size_t bfgs_lds_bytes(int lanes);
size_t lbfgs_lds_bytes(int slots);

// Lanes per start of the BFGS kernels for a problem (power of two >= dim, at
// most 64; kTileBlockDim for one block per start with H in registers,
// d <= 128; kHybridDim for one block per start with H in registers and LDS,
// d <= 208; kWideLanes for one block per start with H in device memory), from
// the tiling table.
int group_lanes(int objective, int precision, int dim);

// One rule of the tiling table: problems of this objective and precision
// with dmin <= dim <= dmax run with `lanes` lanes per start.
struct TileRule {
  int objective, precision, dmin, dmax, lanes;
};
// Coordinate slots per particle of the swarm kernels (power of two >= dim;
// lanes per particle are min(slots, 64)), and one request's grid size.
int pso_group_lanes(int dim);
int pso_blocks(int64_t n, int dim);

}  // namespace zeus
