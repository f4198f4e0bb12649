// vegas_rtc.cpp — integrands compiled at run time.
//
// The paper's user writes the integrand as an ordinary function of a batch
// of points (Sec. 3.1). Here the user's device functions are compiled with
// hiprtc together with the library's own iteration kernel: the text of the
// headers the built-in kernels are compiled from is embedded at build time,
// and k_iterate is instantiated with the user's functions as its integrand,
// so a run-time integrand goes through the same draw / map / Jacobian /
// moments / histogram code as the built-in ones. The code object is kept on
// the host and loaded onto a GPU the first time the integrand runs there.
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "vegas.h"
#include "vegas_launch.hpp"
#include "vegas_types.hpp"

namespace vegas {
namespace {

// kRtcKernelSource: vegas_math.hpp, vegas_types.hpp, vegas_device.hpp and
// vegas_iterate.hpp
// with their #include lines blanked (hiprtc supplies the HIP device API).
#include "vegas_rtc_source.inc"

static_assert(VEGAS_F_USER == kUser && VEGAS_MAX_USER == kMaxUser &&
                  VEGAS_MAX_USER_PARAMS == kUserParams,
              "run-time integrand limits");

// The fixed-width integer names the kernel headers use; hiprtc has them only
// in its internal namespace.
const char kPrelude[] =
    "typedef __hip_internal::uint32_t uint32_t;\n"
    "typedef __hip_internal::uint64_t uint64_t;\n"
    "typedef __hip_internal::int32_t int32_t;\n"
    "typedef __hip_internal::int64_t int64_t;\n";

// The integrand type k_iterate is instantiated with.
const char kWrapper[] =
    "\n#line 1 \"vegas_user_integrand\"\n"
    "struct vegas_user_integrand {\n"
    "  static __device__ __forceinline__ double f64(const double* x, int d, const double* p) {\n"
    "    return vegas_user_f64(x, d, p);\n"
    "  }\n"
    "  static __device__ __forceinline__ float f32(const float* x, int d, const float* p) {\n"
    "    return vegas_user_f32(x, d, p);\n"
    "  }\n"
    "};\n";

const char* const kOptions[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-munsafe-fp-atomics",
    // no packed FP32 instructions, as for the library's own kernels
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};

// Template dimension argument of k_iterate for `dim` dimensions: the exact
// count up to 16, else the class of 20/24/28/32 (as for the built-in kernels).
int dims_arg(int dim) {
  if (dim <= 16) return dim;
  return -(((dim + 3) / 4) * 4);
}

struct UserIntegrand {
  int dim = 0;                       // 0: any dimension
  std::vector<int> classes;          // template dimension arguments compiled
  std::vector<char> code;            // code object for gfx950
  std::vector<std::string> lowered;  // kernel names, index variant(class, prec, dump)
  struct Loaded {
    hipModule_t mod = nullptr;
    std::vector<hipFunction_t> fn;
  };
  std::map<int, Loaded> loaded;  // by device
};

int variant(int cls, int prec, bool dump) { return (cls * 2 + prec) * 2 + (dump ? 1 : 0); }

std::mutex g_mu;
std::vector<std::unique_ptr<UserIntegrand>> g_user;

void put_log(char* log, size_t log_bytes, const std::string& s) {
  if (!log || log_bytes == 0) return;
  const size_t n = s.size() < log_bytes - 1 ? s.size() : log_bytes - 1;
  std::memcpy(log, s.data(), n);
  log[n] = '\0';
}

// Dimension-class index of a handle of `dim` dimensions; -1 if none.
int class_of(const UserIntegrand& u, int dim) {
  if (u.dim) return dim == u.dim ? 0 : -1;
  return dim <= 16 ? 0 : 1;
}

}  // namespace

int user_integrand_fits(int fid, int dim) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int i = fid - kUser;
  if (i < 0 || i >= (int)g_user.size() || dim < 1 || dim > kMaxDim) return 0;
  return class_of(*g_user[i], dim) >= 0;
}

IterKernel user_iterate_kernel(int fid, int prec, int dim, bool dump) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int i = fid - kUser;
  if (i < 0 || i >= (int)g_user.size() || dim < 1 || dim > kMaxDim ||
      (prec != kFp64 && prec != kFp32Eval))
    return IterKernel{};
  UserIntegrand& u = *g_user[i];
  const int cls = class_of(u, dim);
  if (cls < 0) return IterKernel{};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return IterKernel{};
  auto it = u.loaded.find(dev);
  if (it == u.loaded.end()) {
    UserIntegrand::Loaded L;
    if (hipModuleLoadData(&L.mod, u.code.data()) != hipSuccess) return IterKernel{};
    L.fn.resize(u.lowered.size());
    for (size_t v = 0; v < u.lowered.size(); ++v)
      if (hipModuleGetFunction(&L.fn[v], L.mod, u.lowered[v].c_str()) != hipSuccess) {
        (void)hipModuleUnload(L.mod);
        return IterKernel{};
      }
    it = u.loaded.emplace(dev, std::move(L)).first;
  }
  IterKernel k;
  k.mf = it->second.fn[variant(cls, prec, dump)];
  return k;
}

}  // namespace vegas

using namespace vegas;

extern "C" int vegas_integrand_compile(const char* source, int dim, int* integrand_id, char* log,
                                       size_t log_bytes) {
  if (!source || !integrand_id || dim < 0 || dim > kMaxDim) return VEGAS_EINVAL;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_user.size() >= kMaxUser) return VEGAS_ENOMEM;
  }
  auto u = std::make_unique<UserIntegrand>();
  u->dim = dim;
  if (dim)
    u->classes = {dims_arg(dim)};
  else
    u->classes = {-16, -32};

  std::string src = kPrelude;
  src += reinterpret_cast<const char*>(kRtcKernelSource);
  src += "\n#line 1 \"integrand.hip\"\n";
  src += source;
  src += kWrapper;

  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "vegas_user.hip", 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS)
    return VEGAS_ENOMEM;
  std::vector<std::string> names;
  for (size_t c = 0; c < u->classes.size(); ++c)
    for (int prec = 0; prec < 2; ++prec)
      for (int dump = 0; dump < 2; ++dump) {
        char buf[128];
        std::snprintf(buf, sizeof(buf), "vegas::k_iterate<%d, %d, %d, %s, vegas_user_integrand>",
                      u->classes[c], kUser, prec, dump ? "true" : "false");
        names.emplace_back(buf);
      }
  for (const std::string& n : names) hiprtcAddNameExpression(prog, n.c_str());
  const hiprtcResult rc = hiprtcCompileProgram(
      prog, (int)(sizeof(kOptions) / sizeof(kOptions[0])), kOptions);
  if (rc != HIPRTC_SUCCESS) {
    size_t n = 0;
    std::string text;
    if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 0) {
      text.resize(n);
      if (hiprtcGetProgramLog(prog, &text[0]) != HIPRTC_SUCCESS) text.clear();
    }
    if (text.empty()) text = hiprtcGetErrorString(rc);
    put_log(log, log_bytes, text);
    hiprtcDestroyProgram(&prog);
    return VEGAS_ECOMPILE;
  }
  size_t code_bytes = 0;
  bool ok = hiprtcGetCodeSize(prog, &code_bytes) == HIPRTC_SUCCESS && code_bytes > 0;
  if (ok) {
    u->code.resize(code_bytes);
    ok = hiprtcGetCode(prog, u->code.data()) == HIPRTC_SUCCESS;
  }
  for (size_t i = 0; ok && i < names.size(); ++i) {
    const char* lowered = nullptr;
    ok = hiprtcGetLoweredName(prog, names[i].c_str(), &lowered) == HIPRTC_SUCCESS && lowered;
    if (ok) u->lowered.emplace_back(lowered);
  }
  hiprtcDestroyProgram(&prog);
  if (!ok) {
    put_log(log, log_bytes, "hiprtc produced no code object");
    return VEGAS_ECOMPILE;
  }
  put_log(log, log_bytes, "");
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_user.size() >= kMaxUser) return VEGAS_ENOMEM;
  *integrand_id = kUser + (int)g_user.size();
  g_user.push_back(std::move(u));
  return VEGAS_OK;
}
