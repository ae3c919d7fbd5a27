// zeus_bfgs_tile.hip -- launches of the on-chip block kernel for 64 < d <= 128
// (the kernel template is in zeus_bfgs_tile_kernels.h).
#include "zeus_bfgs_tile_kernels.h"

namespace zeus {
namespace {

// The kernel is persistent: as many blocks as can be resident at once.
template <int OBJ, class T>
hipError_t launch_tile_t(const Group &g, int cus) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&bfgs_tile_kernel<OBJ, T>), kBlockLanes, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t cap = (int64_t)cus * per_cu;
  if (g.resident) {
    *g.resident = cap;
    return hipSuccess;
  }
  const int blocks = (int)(g.total_starts < cap ? g.total_starts : cap);
  hipLaunchKernelGGL((bfgs_tile_kernel<OBJ, T>), dim3(blocks), dim3(kBlockLanes), 0, g.stream,
                     g.reqs, g.nreq, g.hdr, g.total_starts);
  return hipGetLastError();
}

template <class T>
hipError_t launch_tile_prec(const Group &g, int cus) {
  switch (g.objective) {
    case kRosenbrock: return launch_tile_t<kRosenbrock, T>(g, cus);
    case kRastrigin: return launch_tile_t<kRastrigin, T>(g, cus);
    case kAckley: return launch_tile_t<kAckley, T>(g, cus);
    case kStyblinskiTang: return launch_tile_t<kStyblinskiTang, T>(g, cus);
    case kSphere: return launch_tile_t<kSphere, T>(g, cus);
    case kQuartic: return launch_tile_t<kQuartic, T>(g, cus);
    default: return hipErrorInvalidValue;  // Goldstein-Price has d == 2
  }
}

}  // namespace

hipError_t launch_bfgs_tile(const Group &g, int cus) {
  if (g.precision == ZEUS_MIXED) return launch_tile_prec<float>(g, cus);
  return launch_tile_prec<double>(g, cus);
}

}  // namespace zeus
