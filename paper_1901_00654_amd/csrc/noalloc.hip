// ts_solve_noalloc: the whole smoothing solve (ts_create + ts_solve) with
// every device buffer carved from one file-scope device array, for callers
// that cannot allocate device memory. The array is reached through the
// address hipGetSymbolAddress reports for it on each device (host code never
// passes the symbol itself to a kernel or a copy).
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "api_util.h"
#include "problem.h"

namespace tsmg {
namespace {

constexpr size_t kScratchBytes = size_t(TS_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
  std::mutex call;        // one solve at a time per device
  void* ptr = nullptr;    // device address of `scratch` on this device
};

std::mutex g_init;
DeviceScratch g_dev[kMaxDevices];

// Device address of the scratch array on the current device, looked up once.
DeviceScratch& device_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error{TS_EDEVICE, "device index out of range"};
  std::lock_guard<std::mutex> lk(g_init);
  DeviceScratch& D = g_dev[dev];
  if (!D.ptr) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw Error{TS_EDEVICE, "no device address for the scratch array"};
    register_arena_region(p, kScratchBytes);
    D.ptr = p;
  }
  return D;
}

thread_local std::vector<double> t_history;

struct ArenaScope {
  Arena a;
  explicit ArenaScope(void* base) {
    a.base = static_cast<char*>(base);
    a.cap = kScratchBytes;
    a.used = 0;
    g_arena = &a;
  }
  ~ArenaScope() { g_arena = nullptr; }
};

}  // namespace
}  // namespace tsmg

extern "C" {

ts_status ts_solve_noalloc(int d, int q, const int32_t* intervals, const double* lo, const double* hi, int64_t n,
                           const double* x, const double* y, double lambda, const ts_options* opt, double* alpha,
                           ts_solve_info* info) {
  TS_API_BEGIN
  if (q != 3) throw tsmg::Error{TS_EINVAL, "only cubic splines (q = 3) are supported"};
  if (!alpha) throw tsmg::Error{TS_EINVAL, "alpha must not be null"};
  if (d < 1 || d > tsmg::kMaxDim || !intervals) throw tsmg::Error{TS_EINVAL, "d must be in 1..5"};
  if (intervals[0] < 2 || intervals[0] > (1 << 20)) throw tsmg::Error{TS_EINVAL, "intervals out of range"};
  if (tsmg::needs_general(d, q, intervals, opt ? opt->degrees : nullptr))
    throw tsmg::Error{TS_EINVAL, "the no-allocation solve takes cubic splines on equal power-of-two grids"};
  int dev = 0;
  tsmg::hip_check(hipGetDevice(&dev), "hipGetDevice");
  tsmg::DeviceScratch& D = tsmg::device_scratch(dev);
  ts_options o;
  ts_default_options(&o);
  if (opt) o = *opt;
  o.bottom_max_k = -1;   // every V-cycle level runs its own steps (no dense operator to assemble)
  // reject sizes beyond the scratch before any work: the estimate of the
  // peak bytes with stencils held to half of the scratch
  {
    const int64_t need = tsmg::footprint_bytes(d, intervals[0], n, o, 0.5 * double(tsmg::kScratchBytes));
    if (need > int64_t(tsmg::kScratchBytes))
      throw tsmg::Error{TS_EINVAL, "problem needs about " + std::to_string(need) + " bytes of device memory, more "
                                   "than the " + std::to_string(tsmg::kScratchBytes) + "-byte no-allocation scratch"};
  }
  std::lock_guard<std::mutex> lk(D.call);
  tsmg::ArenaScope scope(D.ptr);
  std::unique_ptr<tsmg::Problem> P(tsmg::create_problem(d, q, intervals, lo, hi, n, x, y, lambda, &o));
  ts_solve_info inf{};
  const ts_status s = tsmg::solve(P.get(), alpha, 0, &inf);
  tsmg::t_history = P->history;
  inf.residual_history = tsmg::t_history.data();
  inf.history_len = int(tsmg::t_history.size());
  P.reset();   // synchronises the stream before the scratch is handed to the next call
  if (info) *info = inf;
  return s;
  TS_API_END
}

}  // extern "C"
