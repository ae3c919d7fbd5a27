// zeus_user.cpp -- user objectives: run-time compilation of the kernel
// templates with the user's source (hipRTC) and their launches.
//
// The program is zeus_user.h, the user's source, zeus_user_elem.h and the
// swarm, BFGS and L-BFGS kernel templates, instantiated for kUser at every
// size (swarm: 2..256 coordinate slots per particle, one per lane up to 64
// lanes and 2 or 4 per lane beyond; BFGS: 4..64 lanes per start, and the two
// on-chip block kernels for 64 < d <= 128 and <= 208; L-BFGS: 4..256
// coordinate slots per start; the BFGS and L-BFGS kernels in FP64 and in
// mixed precision).  The
// headers are compiled into the library as text (zeus_rtc_headers.inc,
// generated from the sources by the build), so the same template code runs
// for built-in and user objectives.  The build's code-generation flags are
// passed to hipRTC.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <string>
#include <vector>

#include "zeus_internal.h"

namespace zeus {
namespace {

struct RtcHeader {
  const char *name, *text;
};
#include "zeus_rtc_headers.inc"  // kRtcHeaders[], kRtcHeaderCount

// System headers the kernel headers include, reduced to what device code
// needs (the host declarations in zeus_internal.h only need the type names).
const RtcHeader kRtcStubs[] = {
    {"hip/hip_runtime.h",
     "#pragma once\ntypedef struct ihipStream_t *hipStream_t;\ntypedef int hipError_t;\n"},
    {"stdint.h",
     "#pragma once\ntypedef __INT8_TYPE__ int8_t;\ntypedef __INT16_TYPE__ int16_t;\n"
     "typedef __INT32_TYPE__ int32_t;\ntypedef __INT64_TYPE__ int64_t;\n"
     "typedef __UINT8_TYPE__ uint8_t;\ntypedef __UINT16_TYPE__ uint16_t;\n"
     "typedef __UINT32_TYPE__ uint32_t;\ntypedef __UINT64_TYPE__ uint64_t;\n"
     "#define INT64_MAX __INT64_MAX__\n"},
    {"stddef.h", "#pragma once\ntypedef __SIZE_TYPE__ size_t;\ntypedef __PTRDIFF_TYPE__ ptrdiff_t;\n"},
};

int log2_of(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

// Compiles `source` for `arch` and, when `out` is given, loads the kernels on
// the current device into *out.  Returns 0, or 1 with the compiler's log in
// *log when the program does not compile, or 2 with a message when a HIP or
// hipRTC call fails.
int user_compile(const char *arch, const char *source, UserKernels *out, std::string *log) {
  UserKernels unused;
  const bool load = out != nullptr;
  if (!out) out = &unused;
  *out = UserKernels{};
  std::string prog;
  prog += "#include \"zeus_user.h\"\n";
  prog += "#line 1 \"objective\"\n";
  prog += source;
  prog += "\n#include \"zeus_user_elem.h\"\n#include \"zeus_pso_kernels.h\"\n"
          "#include \"zeus_bfgs_kernels.h\"\n#include \"zeus_lbfgs_kernels.h\"\n"
          "#include \"zeus_bfgs_tile_kernels.h\"\n#include \"zeus_bfgs_hybrid_kernels.h\"\n";
  std::vector<const char *> names, texts;
  for (int i = 0; i < kRtcHeaderCount; ++i) {
    names.push_back(kRtcHeaders[i].name);
    texts.push_back(kRtcHeaders[i].text);
  }
  for (const RtcHeader &h : kRtcStubs) {
    names.push_back(h.name);
    texts.push_back(h.text);
  }
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, prog.c_str(), "zeus_user_objective.hip", (int)names.size(), texts.data(),
                          names.data()) != HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return 2;
  }
  // slots 2^l as lanes x coordinates per lane
  auto split = [](int l) {
    const int s = 1 << l, lanes = s < 64 ? s : 64;
    return std::to_string(lanes) + ", " + std::to_string(s / lanes);
  };
  std::vector<std::string> pso_expr, bfgs_expr, lbfgs_expr, block_expr;
  for (int l = 1; l <= 8; ++l) pso_expr.push_back("&zeus::pso_kernel<7, " + split(l) + ">");
  // per precision (FP64, then mixed with FP32 evaluations): BFGS 4..64
  // lanes, L-BFGS 4..256 slots, the two block kernels
  for (const char *t : {"double", "float"}) {
    for (int l = 2; l <= 6; ++l)
      bfgs_expr.push_back("&zeus::bfgs_kernel<7, " + std::to_string(1 << l) + ", " + t + ">");
    for (int l = 2; l <= 8; ++l) lbfgs_expr.push_back("&zeus::lbfgs_kernel<7, " + split(l) + ", " + t + ">");
    block_expr.push_back(std::string("&zeus::bfgs_tile_kernel<7, ") + t + ">");
    block_expr.push_back(std::string("&zeus::bfgs_hybrid_kernel<7, ") + t + ">");
  }
  for (const auto *v : {&pso_expr, &bfgs_expr, &lbfgs_expr, &block_expr})
    for (const std::string &e : *v) hiprtcAddNameExpression(p, e.c_str());
  const std::string arch_opt = std::string("--offload-arch=") + arch;
  const char *opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult cr = hiprtcCompileProgram(p, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(p, &ls);
  std::string lg(ls, '\0');
  if (ls) hiprtcGetProgramLog(p, &lg[0]);
  if (cr != HIPRTC_SUCCESS) {
    *log = lg;
    hiprtcDestroyProgram(&p);
    return 1;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(p, &cs);
  std::vector<char> code(cs);
  hiprtcGetCode(p, code.data());
  auto lowered = [&](const std::vector<std::string> &exprs) {
    std::vector<std::string> out_names;
    for (auto &e : exprs) {
      const char *n = nullptr;
      hiprtcGetLoweredName(p, e.c_str(), &n);
      out_names.push_back(n ? n : "");
    }
    return out_names;
  };
  const std::vector<std::string> pso_names = lowered(pso_expr), bfgs_names = lowered(bfgs_expr),
                                 lbfgs_names = lowered(lbfgs_expr), block_names = lowered(block_expr);
  hiprtcDestroyProgram(&p);
  if (!load) return 0;
  hipModule_t mod;
  hipError_t he = hipModuleLoadData(&mod, code.data());
  if (he != hipSuccess) {
    *log = std::string("hipModuleLoadData: ") + hipGetErrorString(he);
    return 2;
  }
  out->module = mod;
  for (int l = 1; l <= 8; ++l) {
    hipFunction_t f;
    if ((he = hipModuleGetFunction(&f, mod, pso_names[l - 1].c_str())) != hipSuccess) break;
    out->pso[l] = f;
  }
  for (int pr = 0; pr < 2; ++pr) {
    for (int l = 2; he == hipSuccess && l <= 6; ++l) {
      hipFunction_t f;
      if ((he = hipModuleGetFunction(&f, mod, bfgs_names[5 * pr + l - 2].c_str())) != hipSuccess) break;
      out->bfgs[pr][l] = f;
    }
    for (int l = 2; he == hipSuccess && l <= 8; ++l) {
      hipFunction_t f;
      if ((he = hipModuleGetFunction(&f, mod, lbfgs_names[7 * pr + l - 2].c_str())) != hipSuccess) break;
      out->lbfgs[pr][l] = f;
    }
    for (int b = 0; he == hipSuccess && b < 2; ++b) {
      hipFunction_t f;
      if ((he = hipModuleGetFunction(&f, mod, block_names[2 * pr + b].c_str())) != hipSuccess) break;
      (b == 0 ? out->bfgs_tile : out->bfgs_hybrid)[pr] = f;
    }
  }
  if (he != hipSuccess) {
    *log = std::string("hipModuleGetFunction: ") + hipGetErrorString(he);
    (void)hipModuleUnload(mod);
    *out = UserKernels{};
    return 2;
  }
  return 0;
}

void user_release(UserKernels *k) {
  if (k->module) (void)hipModuleUnload(static_cast<hipModule_t>(k->module));
  *k = UserKernels{};
}

hipError_t launch_user_pso(const Group &g, int t) {
  const int l = log2_of(g.g_pso);
  if (!g.user || l < 1 || l > 8 || !g.user->pso[l]) return hipErrorInvalidValue;
  const ReqDev *reqs = g.reqs;
  int nreq = g.nreq;
  void *args[] = {&reqs, &nreq, &t};
  return hipModuleLaunchKernel(static_cast<hipFunction_t>(g.user->pso[l]), (unsigned)g.pso_grid, 1, 1,
                               (unsigned)pso_threads(g.g_pso), 1, 1, 0, g.stream, args, nullptr);
}

hipError_t launch_user_bfgs(const Group &g, int64_t want, int cus) {
  const int pr = g.precision == ZEUS_MIXED ? 1 : 0;
  if (g.g_bfgs == kTileBlockDim || g.g_bfgs == kHybridDim) {
    // one block per start, as many as can be resident (static LDS only)
    void *fn = g.user ? (g.g_bfgs == kTileBlockDim ? g.user->bfgs_tile : g.user->bfgs_hybrid)[pr] : nullptr;
    if (!fn) return hipErrorInvalidValue;
    hipFunction_t f = static_cast<hipFunction_t>(fn);
    const int threads = g.g_bfgs == kTileBlockDim ? kWideLanes : 2 * kWideLanes;
    int per_cu = 0;
    hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, threads, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int64_t cap = (int64_t)cus * per_cu;
    if (g.resident) {
      *g.resident = cap;
      return hipSuccess;
    }
    const unsigned blocks = (unsigned)(g.total_starts < cap ? g.total_starts : cap);
    const ReqDev *reqs = g.reqs;
    int nreq = g.nreq;
    BatchDev *hdr = g.hdr;
    int64_t total = g.total_starts;
    void *args[] = {&reqs, &nreq, &hdr, &total};
    return hipModuleLaunchKernel(f, blocks, 1, 1, (unsigned)threads, 1, 1, 0, g.stream, args, nullptr);
  }
  const int l = log2_of(g.g_bfgs);
  if (!g.user || l < 2 || l > 6 || !g.user->bfgs[pr][l]) return hipErrorInvalidValue;
  hipFunction_t f = static_cast<hipFunction_t>(g.user->bfgs[pr][l]);
  const size_t lds = bfgs_lds_bytes(g.g_bfgs);
  int per_cu = 0;
  hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBfgsBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t cap = (int64_t)cus * per_cu;
  if (g.resident) {
    *g.resident = cap * (kBfgsBlock / g.g_bfgs);
    return hipSuccess;
  }
  const unsigned blocks = (unsigned)(want < cap ? want : cap);
  const ReqDev *reqs = g.reqs;
  int nreq = g.nreq;
  BatchDev *hdr = g.hdr;
  int64_t total = g.total_starts;
  void *args[] = {&reqs, &nreq, &hdr, &total};
  return hipModuleLaunchKernel(f, blocks, 1, 1, kBfgsBlock, 1, 1, (unsigned)lds, g.stream, args, nullptr);
}

// The persistent L-BFGS kernel of `g.g_bfgs` coordinate slots: as many
// blocks as can be resident, at most one group per start.
hipError_t launch_user_lbfgs(const Group &g, int cus) {
  const int l = log2_of(g.g_bfgs);
  const int pr = g.precision == ZEUS_MIXED ? 1 : 0;
  if (!g.user || l < 2 || l > 8 || (1 << l) != g.g_bfgs || !g.user->lbfgs[pr][l])
    return hipErrorInvalidValue;
  hipFunction_t f = static_cast<hipFunction_t>(g.user->lbfgs[pr][l]);
  const int lanes = g.g_bfgs < 64 ? g.g_bfgs : 64;
  const size_t lds = lbfgs_lds_bytes(g.g_bfgs);
  int per_cu = 0;
  hipError_t e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBfgsBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int64_t per_block = kBfgsBlock / lanes;
  const int64_t want = (g.total_starts + per_block - 1) / per_block;
  const int64_t cap = (int64_t)cus * per_cu;
  if (g.resident) {
    *g.resident = cap * per_block;
    return hipSuccess;
  }
  const unsigned blocks = (unsigned)(want < cap ? want : cap);
  const ReqDev *reqs = g.reqs;
  int nreq = g.nreq;
  BatchDev *hdr = g.hdr;
  int64_t total = g.total_starts;
  void *args[] = {&reqs, &nreq, &hdr, &total};
  return hipModuleLaunchKernel(f, blocks, 1, 1, kBfgsBlock, 1, 1, (unsigned)lds, g.stream, args, nullptr);
}

}  // namespace zeus
