// dash_init_noalloc: the initial decomposition of dash_init with its device
// workspace in a fixed, file-scope array instead of a per-call hipMalloc, for
// callers that cannot allocate device memory.
//
// The array is a device symbol: each GPU the library runs on holds its own
// copy (kScratchBytes, until the process ends).  In host code its name is only
// a stand-in, so its device address is looked up once per device with
// hipGetSymbolAddress and kept; the kernels get that address.  The call is
// synchronous and every call on a GPU uses that GPU's array, so calls that
// overlap on one GPU (from several threads) race.  Every workspace word the
// kernels read is written by them earlier in the same call: nothing needs
// clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dash_ctx.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

double *g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device
std::mutex g_mu;

// The device address of this GPU's scratch (looked up on first use).
dash_status scratch_on(int device, double **out) {
  if (device < 0 || device >= kMaxDevices) return DASH_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return DASH_E_DEVICE;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) return DASH_E_DEVICE;
    g_scratch[device] = (double *)p;
  }
  *out = g_scratch[device];
  return DASH_OK;
}

}  // namespace

extern "C" {

size_t dash_init_noalloc_limit(void) { return kScratchBytes; }

dash_status dash_init_noalloc(dash_ctx *c, int32_t K, const int64_t *row_ptr, const float *X, const float *V0,
                              dash_init_report *report) {
  if (c && row_ptr && dash::on_device(row_ptr))
    return dash::fail(c, DASH_E_INVALID_ARG, "dash_init_noalloc takes row_ptr in host memory");
  if (dash_status s = dash::init_check(c, K, row_ptr, X)) return s;
  const size_t need = dash::init_workspace_doubles(c, K, V0 != nullptr);
  if (need > kScratchDoubles)
    return dash::fail(c, DASH_E_CAPACITY,
                      "dash_init_noalloc: the workspace (%zu bytes for J=%d, R=%d, K=%d%s) exceeds its fixed %zu bytes",
                      need * sizeof(double), c->J, c->R, K, V0 ? "" : ", no V0", kScratchBytes);
  double *ws = nullptr;
  if (dash_status s = scratch_on(c->cfg.device, &ws))
    return dash::fail(c, s, "dash_init_noalloc: no address for the scratch array on device %d", c->cfg.device);
  const dash_status s = dash::init_with_workspace(c, K, row_ptr, X, V0, report, ws);
  // the array is free for the next call only once this one's kernels are done
  if (s != DASH_OK) (void)hipStreamSynchronize(c->stream);
  return s;
}

}  // extern "C"
