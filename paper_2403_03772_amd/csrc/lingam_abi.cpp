// C ABI of the library (declared in include/lingam.h): argument validation,
// workspace planning and the host-side step loop that enqueues the kernels.
//
// Control crosses the host/device boundary once per call.  The host knows the
// number of active variables at every step (m = d - t), so it can enqueue the
// whole ordering up front; the identity of each step's chosen variable lives
// only on the device (in the workspace control block and the active list).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/lingam.h"
#include "lingam_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LINGAM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Largest sizes the kernels' 32-bit sample/variable indexing supports.
constexpr int64_t kMaxD = 32768;
constexpr int64_t kMaxN = (int64_t)1 << 30;

struct DevInfo {
  int num_cu = 0;
};

std::mutex g_mu;
std::vector<DevInfo> g_dev;

int num_cu_of_current(int* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  if (g_dev[dev].num_cu == 0) {
    int cu = 0;
    e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    g_dev[dev].num_cu = cu > 0 ? cu : 1;
  }
  *out = g_dev[dev].num_cu;
  return LINGAM_OK;
}

int status_from_device(int32_t s) {
  switch (s) {
    case 0:
      return LINGAM_OK;
    case LINGAM_E_INVALID:
      return fail(LINGAM_E_INVALID, "forced_order names a variable that is not active");
    case LINGAM_E_DEGENERATE:
      return fail(LINGAM_E_DEGENERATE,
                  "degenerate data: non-finite value, zero-variance column or collinear pair");
    default:
      return fail(LINGAM_E_HIP, "unexpected device status %d", s);
  }
}

// Event pair recorder for the optional profile.
struct Timer {
  std::vector<hipEvent_t> ev;
  bool on = false;
  int take(hipStream_t st) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    ev.push_back(e);
    (void)hipEventRecord(e, st);
    return (int)ev.size() - 1;
  }
  double ms(int a, int b) {
    float x = 0.f;
    if (a < 0 || b < 0) return 0.0;
    (void)hipEventElapsedTime(&x, ev[a], ev[b]);
    return x;
  }
  ~Timer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

}  // namespace

extern "C" {

void lingam_opts_init(lingam_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(lingam_opts);
}

const char* lingam_last_error(void) { return g_err; }

const char* lingam_version(void) { return "lingam-mi355x 0.1 (gfx950)"; }

size_t lingam_workspace_size(int64_t n, int64_t d, const lingam_opts* opts) {
  (void)opts;
  if (n < 2 || d < 1 || n > kMaxN || d > kMaxD) return 0;
  int cu = 0;
  if (num_cu_of_current(&cu) != LINGAM_OK) cu = 256;
  return lg::make_layout(n, d, cu).total;
}

int lingam_causal_order(const float* X, int64_t n, int64_t d, int64_t ldx, int32_t* order,
                        const lingam_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  lingam_opts dflt;
  lingam_opts_init(&dflt);
  if (!opts) opts = &dflt;
  if (opts->struct_size != sizeof(lingam_opts))
    return fail(LINGAM_E_INVALID, "opts->struct_size %u != %zu", opts->struct_size,
                sizeof(lingam_opts));
  if (!X || !order) return fail(LINGAM_E_INVALID, "X and order must be non-NULL");
  if (n < 2) return fail(LINGAM_E_INVALID, "need n >= 2 samples (got %lld)", (long long)n);
  if (d < 1) return fail(LINGAM_E_INVALID, "need d >= 1 variables (got %lld)", (long long)d);
  if (ldx < d) return fail(LINGAM_E_INVALID, "ldx (%lld) < d (%lld)", (long long)ldx, (long long)d);
  if (n > kMaxN || d > kMaxD)
    return fail(LINGAM_E_UNSUPPORTED, "n <= %lld and d <= %lld supported", (long long)kMaxN,
                (long long)kMaxD);
  if (opts->forced_len < 0 || opts->forced_len > d)
    return fail(LINGAM_E_INVALID, "forced_len %d outside [0, d]", opts->forced_len);
  if (opts->forced_len > 0 && !opts->forced_order)
    return fail(LINGAM_E_INVALID, "forced_len > 0 but forced_order is NULL");
  int cu = 0;
  int rc = num_cu_of_current(&cu);
  if (rc != LINGAM_OK) return rc;
  const lg::Layout L = lg::make_layout(n, d, cu);
  if (!ws || ws_bytes < L.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", L.total,
                ws ? ws_bytes : (size_t)0);

  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  Timer tm;
  tm.on = opts->profile != nullptr;
  int ev_all0 = tm.on ? tm.take(st) : -1;
  hipError_t e;
#define LG_TRY(call, what)                    \
  do {                                        \
    e = (call);                               \
    if (e != hipSuccess) return hip_fail(e, what); \
  } while (0)

  LG_TRY(lg::launch_init(L, w, order, st), "init");
  LG_TRY(lg::launch_ingest(L, w, X, ldx, st), "ingest");
  LG_TRY(lg::launch_moments(L, w, st), "moments");
  int ev_g0 = tm.on ? tm.take(st) : -1;
  LG_TRY(lg::launch_gram(L, w, st), "gram");
  int ev_g1 = tm.on ? tm.take(st) : -1;
  LG_TRY(lg::launch_standardize(L, w, st), "standardize");

  std::vector<int> pair_ev, resid_ev;
  double pair_evals = 0.0, resid_bytes = 0.0;
  const int forced_len = opts->forced_len;
  for (int64_t t = 0; t + 1 < d; ++t) {
    const int m = (int)(d - t);
    if (m > lg::kFp64MaxM) {
      const lg::StepPlan p = lg::plan_step(m, L.n_pad, cu);
      if (tm.on) pair_ev.push_back(tm.take(st));
      LG_TRY(lg::launch_pair(L, w, m, p, st), "pair");
      if (tm.on) pair_ev.push_back(tm.take(st));
      pair_evals += (double)m * (double)(m - 1) * (double)n;
      LG_TRY(lg::launch_combine(L, w, m, p, st), "combine");
    } else {
      LG_TRY(lg::launch_pair64(L, w, m, st), "pair64");
    }
    LG_TRY(lg::launch_rowk(L, w, m, st), "rowk");
    LG_TRY(lg::launch_select(L, w, m, (int)t, order, opts->forced_order, forced_len,
                             opts->step_measures, opts->step_gap, st),
           "select");
    if (m > 2) {
      if (tm.on) resid_ev.push_back(tm.take(st));
      LG_TRY(lg::launch_resid(L, w, m - 1, st), "resid");
      if (tm.on) resid_ev.push_back(tm.take(st));
      resid_bytes += 28.0 * (double)n * (double)(m - 1);
    }
  }
  if (opts->dev_status) LG_TRY(lg::launch_copy_status(L, w, opts->dev_status, st), "status");
  int ev_all1 = tm.on ? tm.take(st) : -1;
#undef LG_TRY

  const bool sync = !(opts->flags & LINGAM_FLAG_NO_SYNC) || tm.on;
  if (!sync) return LINGAM_OK;
  int32_t dev_status = 0;
  e = hipMemcpyAsync(&dev_status, w + L.ctrl, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(status)");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (tm.on) {
    lingam_profile* pr = opts->profile;
    memset(pr, 0, sizeof(*pr));
    pr->total_ms = tm.ms(ev_all0, ev_all1);
    pr->gram_ms = tm.ms(ev_g0, ev_g1);
    pr->gram_flops = 2.0 * (double)n * (double)d * (double)d;
    for (size_t k = 0; k + 1 < pair_ev.size(); k += 2) pr->pair_ms += tm.ms(pair_ev[k], pair_ev[k + 1]);
    pr->pair_launches = (int64_t)(pair_ev.size() / 2);
    pr->pair_evals = pair_evals;
    for (size_t k = 0; k + 1 < resid_ev.size(); k += 2)
      pr->resid_ms += tm.ms(resid_ev[k], resid_ev[k + 1]);
    pr->resid_bytes = resid_bytes;
  }
  return status_from_device(dev_status);
}

size_t lingam_residualize_workspace_size(int64_t n, int64_t d) {
  if (n < 2 || d < 1 || n > kMaxN || d > kMaxD) return 0;
  return lg::resid_ws_size(n, d);
}

int lingam_residualize(float* X, int64_t n, int64_t d, int64_t ldx, const int32_t* active,
                       int32_t n_active, int32_t exo, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X || !active) return fail(LINGAM_E_INVALID, "X and active must be non-NULL");
  if (n < 2 || d < 1 || ldx < d)
    return fail(LINGAM_E_INVALID, "bad sizes n=%lld d=%lld ldx=%lld", (long long)n,
                (long long)d, (long long)ldx);
  if (n > kMaxN || d > kMaxD) return fail(LINGAM_E_UNSUPPORTED, "size beyond supported range");
  if (n_active < 1 || n_active > d)
    return fail(LINGAM_E_INVALID, "n_active %d outside [1, d]", n_active);
  if (exo < 0 || exo >= d) return fail(LINGAM_E_INVALID, "exo %d outside [0, d)", exo);
  const size_t need = lg::resid_ws_size(n, d);
  if (!ws || ws_bytes < need)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", need,
                ws ? ws_bytes : (size_t)0);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = lg::launch_residualize_rowmajor(X, n, d, ldx, active, n_active, exo, (char*)ws, st);
  if (e != hipSuccess) return hip_fail(e, "residualize launch");
  int32_t s = 0;
  e = hipMemcpyAsync(&s, ws, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(status)");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (s == LINGAM_E_INVALID) return fail(LINGAM_E_INVALID, "an id in `active` is outside [0, d)");
  if (s != 0) return fail(LINGAM_E_DEGENERATE, "var(x_exo) == 0");
  return LINGAM_OK;
}

}  // extern "C"
