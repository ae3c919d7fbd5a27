// zeus_bfgs_hybrid.hip -- launches of the register-and-LDS block kernel for
// 128 < d <= 208 (the kernel template is in zeus_bfgs_hybrid_kernels.h).
#include "zeus_bfgs_hybrid_kernels.h"

namespace zeus {
namespace {

// The kernel is persistent: as many blocks as can be resident at once (one
// per CU: the block holds most of the CU's LDS).
template <int OBJ, class T>
hipError_t launch_hybrid_t(const Group &g, int cus) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&bfgs_hybrid_kernel<OBJ, T>), kHLanes, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;  // the block does not fit a CU
  const int64_t cap = (int64_t)cus * per_cu;
  if (g.resident) {
    *g.resident = cap;
    return hipSuccess;
  }
  const int blocks = (int)(g.total_starts < cap ? g.total_starts : cap);
  hipLaunchKernelGGL((bfgs_hybrid_kernel<OBJ, T>), dim3(blocks), dim3(kHLanes), 0, g.stream,
                     g.reqs, g.nreq, g.hdr, g.total_starts);
  return hipGetLastError();
}

template <class T>
hipError_t launch_hybrid_prec(const Group &g, int cus) {
  switch (g.objective) {
    case kRosenbrock: return launch_hybrid_t<kRosenbrock, T>(g, cus);
    case kRastrigin: return launch_hybrid_t<kRastrigin, T>(g, cus);
    case kAckley: return launch_hybrid_t<kAckley, T>(g, cus);
    case kStyblinskiTang: return launch_hybrid_t<kStyblinskiTang, T>(g, cus);
    case kSphere: return launch_hybrid_t<kSphere, T>(g, cus);
    case kQuartic: return launch_hybrid_t<kQuartic, T>(g, cus);
    default: return hipErrorInvalidValue;  // Goldstein-Price has d == 2
  }
}

}  // namespace

hipError_t launch_bfgs_hybrid(const Group &g, int cus) {
  if (g.precision == ZEUS_MIXED) return launch_hybrid_prec<float>(g, cus);
  return launch_hybrid_prec<double>(g, cus);
}

}  // namespace zeus
