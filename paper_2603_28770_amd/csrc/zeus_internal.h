// zeus_internal.h -- host-side declarations shared by the C-ABI layer and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/zeus.h"

namespace zeus {

// Largest dimension the one-group-per-start kernels handle (a group is at most
// one 64-lane wavefront; lane j owns row j of the inverse Hessian).
constexpr int kMaxDim = 64;
constexpr int kPsoBlock = 256;
constexpr int kBfgsBlock = 256;

// Most blocks a swarm launch uses (the grid strides over the particles; every
// block re-reduces the previous launch's P block results, so P stays small).
constexpr int kPsoMaxBlocks = 512;

// A swarm best, kept on the device.
struct PsoBest {
  double f;      // value as computed (may be NaN if every value is NaN)
  int64_t idx;   // particle index
};

// Device workspace carved out of one allocation (all offsets 256-aligned).
// The swarm kernels exchange their block results through double-buffered
// slots: sweep t writes slot t & 1, sweep t+1 reads it after the kernel
// boundary, so no launch needs a device-wide fence.
struct Workspace {
  uint64_t *queue;         // next unclaimed BFGS start
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
  int pso_blocks;          // P
};

size_t workspace_bytes(int64_t n, int dim);
Workspace carve_workspace(void *base, int64_t n, int dim);

struct Launch {
  const zeus_problem *pb;
  const zeus_result *out;  // device pointers
  Workspace ws;
  hipStream_t stream;
};

// Kernel launchers (return the first HIP error, hipSuccess otherwise).
hipError_t launch_ws_init(const Launch &L);
hipError_t launch_pso_init(const Launch &L);
hipError_t launch_pso_step(const Launch &L, int t);
hipError_t launch_pso_finish(const Launch &L);
hipError_t launch_bfgs(const Launch &L);
hipError_t launch_summary(const Launch &L);

// Lanes per start of the BFGS kernel for a dimension (power of two >= dim).
int group_lanes(int dim);
// Lanes per particle of the swarm kernels, and their grid size.
int pso_group_lanes(int dim);
int pso_blocks(int64_t n, int dim);

}  // namespace zeus
