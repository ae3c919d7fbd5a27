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

// Global best of the swarm, kept on the device.
struct PsoBest {
  double f;      // value as computed (may be NaN if every value is NaN)
  int64_t idx;   // particle index
};

// Device workspace carved out of one allocation (all offsets 256-aligned).
struct Workspace {
  uint32_t *pso_counter;   // blocks finished in the current PSO launch
  uint64_t *queue;         // next unclaimed BFGS start
  PsoBest *best;           // swarm global best
  double *partial_key;     // [pso_blocks] per-block best keys
  int64_t *partial_idx;    // [pso_blocks]
  double *gx;              // [dim] global-best position
  double *x, *v, *px;      // [n][dim]
  double *pf;              // [n]
  int pso_blocks;
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
hipError_t launch_pso_export(const Launch &L);
hipError_t launch_bfgs(const Launch &L);
hipError_t launch_summary(const Launch &L);

// Lanes per start chosen for a dimension (power of two >= dim, at least 8).
int group_lanes(int dim);

}  // namespace zeus
