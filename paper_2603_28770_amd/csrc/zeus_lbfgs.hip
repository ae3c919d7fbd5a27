// zeus_lbfgs.hip -- limited-memory BFGS on gfx950: the launches (the
// kernel template is in zeus_lbfgs_kernels.h).
#include "zeus_lbfgs_kernels.h"

namespace zeus {
namespace {

template <int OBJ, int G, int CPL, class T>
hipError_t launch_l(const Group &g, int cus) {
  const size_t lds = sizeof(double) * (size_t)lbfgs_stride(G * CPL) * (kBfgsBlock / G);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&lbfgs_kernel<OBJ, G, CPL, T>), kBfgsBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t per_block = kBfgsBlock / G;
  const int64_t want = (g.total_starts + per_block - 1) / per_block;
  const int64_t cap = (int64_t)cus * per_cu;
  if (g.resident) {
    *g.resident = cap * per_block;
    return hipSuccess;
  }
  const int blocks = (int)(want < cap ? want : cap);
  hipLaunchKernelGGL((lbfgs_kernel<OBJ, G, CPL, T>), dim3(blocks), dim3(kBfgsBlock), lds, g.stream,
                     g.reqs, g.nreq, g.hdr, g.total_starts);
  return hipGetLastError();
}

template <int OBJ, class T>
hipError_t launch_l_obj(const Group &g, int cus) {
  switch (g.g_bfgs) {  // coordinate slots per start
    case 4: return launch_l<OBJ, 4, 1, T>(g, cus);
    case 8: return launch_l<OBJ, 8, 1, T>(g, cus);
    case 16: return launch_l<OBJ, 16, 1, T>(g, cus);
    case 32: return launch_l<OBJ, 32, 1, T>(g, cus);
    case 64: return launch_l<OBJ, 64, 1, T>(g, cus);
    case 128: return launch_l<OBJ, 64, 2, T>(g, cus);
    case 256: return launch_l<OBJ, 64, 4, T>(g, cus);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t launch_l_prec(const Group &g, int cus) {
  switch (g.objective) {
    case kRosenbrock: return launch_l_obj<kRosenbrock, T>(g, cus);
    case kRastrigin: return launch_l_obj<kRastrigin, T>(g, cus);
    case kAckley: return launch_l_obj<kAckley, T>(g, cus);
    case kStyblinskiTang: return launch_l_obj<kStyblinskiTang, T>(g, cus);
    case kGoldsteinPrice: return launch_l<kGoldsteinPrice, 4, 1, T>(g, cus);
    case kSphere: return launch_l_obj<kSphere, T>(g, cus);
    case kQuartic: return launch_l_obj<kQuartic, T>(g, cus);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t lbfgs_lds_bytes(int slots) {
  const int lanes = slots < 64 ? slots : 64;
  return sizeof(double) * (size_t)lbfgs_stride(slots) * (kBfgsBlock / lanes);
}

int lbfgs_slots(int dim) {
  int s = 4;
  while (s < dim) s <<= 1;
  return s;
}

hipError_t launch_lbfgs(const Group &g, int cus) {
  if (g.objective == kUser) return launch_user_lbfgs(g, cus);
  if (g.precision == ZEUS_MIXED) return launch_l_prec<float>(g, cus);
  return launch_l_prec<double>(g, cus);
}

}  // namespace zeus
