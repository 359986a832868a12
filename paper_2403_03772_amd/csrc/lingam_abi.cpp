// C ABI of the library (declared in include/lingam.h): argument validation,
// workspace planning, the split-policy autotuner, HIP-graph capture, and the
// host-side step loop that enqueues the batched kernels.
//
// Control crosses the host/device boundary once per call.  The host knows the
// number of active variables of every job at every step (m = d - t), so it
// can enqueue (or capture) the whole ordering up front; the identity of each
// step's chosen variable lives only on the device.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lingam.h"
#include "lingam_internal.h"
#include "lingam_linalg.h"

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

#define LG_TRY(call, what)                           \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Largest sizes the kernels' 32-bit sample/variable indexing supports.
constexpr int64_t kMaxD = 32768;
constexpr int64_t kMaxN = (int64_t)1 << 30;
constexpr int kMaxJobs = 65536;

// --------------------------------------------------------------------------
// per-device state: CU count, capture stream, graph cache, autotune cache
// --------------------------------------------------------------------------

struct GraphEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
};

struct DevState {
  int num_cu = 0;
  hipStream_t capture = nullptr;
  std::list<GraphEntry> graphs;  // most recently used first
  std::map<std::string, lg::Tune> tunes;
  bool tunes_loaded = false;
};

std::mutex g_mu;
std::vector<DevState> g_dev;

int current_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_dev.size() <= *dev) g_dev.resize(*dev + 1);
  return LINGAM_OK;
}

int num_cu_of_current(int* out) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc != LINGAM_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_dev[dev].num_cu == 0) {
    int cu = 0;
    hipError_t e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
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
      return fail(LINGAM_E_INVALID,
                  "forced_order names a variable that is not active, or a row index is out "
                  "of range");
    case LINGAM_E_DEGENERATE:
      return fail(LINGAM_E_DEGENERATE,
                  "degenerate data: non-finite value, zero-variance column or collinear pair");
    default:
      return fail(LINGAM_E_HIP, "unexpected device status %d", s);
  }
}

// Event recorder for the optional profile.
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

struct Prof {
  Timer tm;
  std::vector<int> pair_ev, resid_ev, cand_ev;
  int all0 = -1, all1 = -1, g0 = -1, g1 = -1;
  double pair_evals = 0.0, resid_bytes = 0.0, gram_flops = 0.0, cand_evals = 0.0;
};

// --------------------------------------------------------------------------
// batch plan: [job table][schedule][job 0 regions][job 1 regions]...
// --------------------------------------------------------------------------

struct HostJob {
  const float* X;
  const int32_t* rows;
  int64_t n_src, ldx, n, d;
  int32_t* order;
  double* measures;
  double* gaps;
  const int32_t* forced;
  int32_t forced_len;
  float* record = nullptr;  // optional feature record
  int32_t* step_log = nullptr;  // optional per-step decision log (learned form)
};

// Learned-form configuration of a call (proposer == NULL: plain search).
struct Learn {
  const float* proposer = nullptr;
  int32_t K = 0, min_m = 0, audit_every = 0, max_suspects = 0, extension = 0;
  float delta = 0.f;
};

Learn learn_of(const lingam_opts* o) {
  Learn l;
  if (!o || !o->proposer) return l;
  l.proposer = o->proposer;
  l.K = o->topk;
  l.min_m = o->learned_min_m;
  l.audit_every = o->audit_every;
  l.delta = o->margin;
  l.max_suspects = o->max_suspects;
  l.extension = o->extension;
  return l;
}

struct Plan {
  int njobs = 0;
  int cu = 0;
  size_t table_off = 0, sched_off = 0, prop_off = 0, total = 0;
  std::vector<lg::Layout> L;
  std::vector<size_t> job_off;
  int max_d = 0;
  Learn lc;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Plan make_plan(const std::vector<HostJob>& jobs, int cu, const Learn& lc = Learn{}) {
  Plan P;
  P.njobs = (int)jobs.size();
  P.cu = cu;
  P.lc = lc;
  size_t off = 0;
  P.table_off = off;
  off = align256(off + sizeof(lg::JobDev) * (size_t)P.njobs);
  P.sched_off = off;
  off = align256(off + lg::sched_bytes(P.njobs));
  if (lc.proposer) {
    P.prop_off = off;
    off = align256(off + sizeof(lg::PropDev));
  }
  for (const HostJob& j : jobs) {
    P.L.push_back(lg::make_layout(j.n, j.d, cu, lc.proposer ? lc.K : 0));
    P.job_off.push_back(off);
    off = align256(off + P.L.back().total);
    P.max_d = std::max(P.max_d, (int)j.d);
  }
  P.total = off;
  return P;
}

std::vector<lg::JobDev> device_jobs(const Plan& P, const std::vector<HostJob>& jobs, char* ws,
                                    bool tie_on) {
  std::vector<lg::JobDev> out(P.njobs);
  for (int k = 0; k < P.njobs; ++k) {
    const HostJob& h = jobs[k];
    const lg::Layout& L = P.L[k];
    char* b = ws + P.job_off[k];
    lg::JobDev& J = out[k];
    memset(&J, 0, sizeof(J));
    J.X = h.X;
    J.rows = h.rows;
    J.ldx = h.ldx;
    J.n = (int32_t)h.n;
    J.d = (int32_t)h.d;
    J.n_pad = (int32_t)L.n_pad;
    J.ldz = (int32_t)L.ldz;
    J.tie_on = tie_on ? 1 : 0;
    J.tie = reinterpret_cast<int32_t*>(b + L.tie);
    J.tie_r = reinterpret_cast<double*>(b + L.tie_r);
    J.order = h.order;
    J.measures = h.measures;
    J.gaps = h.gaps;
    J.forced = h.forced;
    J.forced_len = h.forced_len;
    J.n_src = (int32_t)std::min<int64_t>(h.n_src, INT32_MAX);
    J.zd = reinterpret_cast<double*>(b + L.zd);
    J.z = reinterpret_cast<float*>(b + L.z);
    J.mu = reinterpret_cast<double*>(b + L.mu);
    J.sig = reinterpret_cast<double*>(b + L.sig);
    J.rho = reinterpret_cast<double*>(b + L.rho);
    J.hm = reinterpret_cast<double*>(b + L.hm);
    J.act = reinterpret_cast<int32_t*>(b + L.act);
    J.ctrl = reinterpret_cast<lg::Ctrl*>(b + L.ctrl);
    J.part = reinterpret_cast<double*>(b + L.part);
    J.rmat = reinterpret_cast<double*>(b + L.rmat);
    J.mvec = reinterpret_cast<double*>(b + L.mvec);
    J.mom = reinterpret_cast<double*>(b + L.mom);
    J.record = h.record;
    if (P.lc.proposer) {
      J.prop = reinterpret_cast<const lg::PropDev*>(ws + P.prop_off);
      J.K = P.lc.K;
      J.min_m = P.lc.min_m;
      J.audit_every = P.lc.audit_every;
      J.delta = P.lc.delta;
      J.feat = reinterpret_cast<float*>(b + L.feat);
      J.score = reinterpret_cast<float*>(b + L.score);
      J.cand = reinterpret_cast<int32_t*>(b + L.cand);
      J.cmark = reinterpret_cast<int32_t*>(b + L.cmark);
      J.partc = reinterpret_cast<double*>(b + L.partc);
      J.rc = reinterpret_cast<double*>(b + L.rc);
      J.kc = reinterpret_cast<double*>(b + L.kc);
      J.lb = reinterpret_cast<double*>(b + L.lb);
      J.wit = reinterpret_cast<int32_t*>(b + L.wit);
      J.ext = reinterpret_cast<int32_t*>(b + L.ext);
      J.ne_max = P.lc.extension;
      J.steplog = h.step_log ? h.step_log : reinterpret_cast<int32_t*>(b + L.steplog);
      J.cap_s = std::min<int32_t>(L.cap_s, P.lc.max_suspects / lg::kTileVars * lg::kTileVars);
      J.cand2 = reinterpret_cast<int32_t*>(b + L.cand2);
      J.parts = reinterpret_cast<double*>(b + L.parts);
      J.rc2 = reinterpret_cast<double*>(b + L.rc2);
      J.kc2 = reinterpret_cast<double*>(b + L.kc2);
    }
  }
  return out;
}

// Host replay of the device schedule: the grid totals of every kernel kind.
struct StepTotals {
  int32_t g[lg::kNumKinds] = {0};
  double pair_evals = 0.0, resid_bytes = 0.0, cand_evals = 0.0;
};

// `ties`: the FP64 resolution of near-ties is on (the learned passes then
// take their own sample splits).
StepTotals step_totals(const std::vector<HostJob>& jobs, const Plan& P, int t, lg::Tune tu,
                       bool ties) {
  StepTotals T;
  std::vector<lg::JobStep> js(P.njobs);
  const int K = P.lc.proposer ? P.lc.K : 0;
  int64_t items = 0, items_c = 0;
  for (int k = 0; k < P.njobs; ++k) {
    js[k] = lg::job_step_base((int32_t)jobs[k].d, t, K, P.lc.min_m, jobs[k].record != nullptr);
    if (js[k].m >= 2 && !js[k].fp64) items += 2LL * js[k].ntiles;
    if (js[k].learned) items_c += 2LL * js[k].nct;
  }
  for (int k = 0; k < P.njobs; ++k) {
    lg::job_split(js[k], (int32_t)P.L[k].n_pad, items, P.cu, tu);
    lg::job_split_cand(js[k], (int32_t)P.L[k].n_pad, items_c, P.cu, tu, ties);
    for (int kind = 0; kind < lg::kNumKinds; ++kind)
      T.g[kind] += lg::kind_count(js[k], kind);
    const int m = js[k].m;
    if (m >= 2 && !js[k].fp64) T.pair_evals += (double)m * (m - 1) * (double)jobs[k].n;
    if (js[k].learned) {
      T.cand_evals += 2.0 * js[k].k * (double)(m - 1) * (double)jobs[k].n;
      // bounds of the suspect pass (its size is decided on the device)
      lg::JobStep b = js[k];
      b.nsus = lg::suspect_cap(
          m, b.k,
          std::min<int32_t>(P.L[k].cap_s, P.lc.max_suspects / lg::kTileVars * lg::kTileVars));
      b.nct2 = lg::cdiv(b.nsus, lg::kTileVars) * b.nblk;
      lg::job_split_susp(b, (int32_t)P.L[k].n_pad, 2LL * b.nct2, P.cu, tu, ties);
      b.ne = lg::ext_count(m, b.k, P.lc.extension);
      b.nct3 = b.ne > 0 ? lg::cdiv(b.nsus, lg::kTileVars) * lg::cdiv(b.ne, lg::kTileVars) : 0;
      for (int kind = lg::kKPairE; kind <= lg::kKLsel2; ++kind)
        T.g[kind] += lg::kind_count(b, kind);
    }
    if (m > 2) T.resid_bytes += 28.0 * (double)jobs[k].n * (double)(m - 1);
  }
  return T;
}

int32_t setup_total(const Plan& P, int kind) {
  int32_t s = 0;
  for (int k = 0; k < P.njobs; ++k)
    s += lg::setup_count((int32_t)P.L[k].n_pad, (int32_t)P.L[k].d, kind);
  return s;
}

// Enqueue the set-up (job table, init, ingest, moments, Gram, standardize).
// `after_gram` runs right after the Gram (VarLiNGAM keeps a copy of rho).
template <typename AfterGram>
int enqueue_setup(const Plan& P, const std::vector<lg::JobDev>& dj, char* ws, hipStream_t st,
                  Prof* pf, AfterGram after_gram) {
  lg::JobDev* table = reinterpret_cast<lg::JobDev*>(ws + P.table_off);
  const lg::SchedDev sc = lg::sched_at(ws + P.sched_off, P.njobs);
  for (int k = 0; k < P.njobs; k += lg::kJobsPerLaunch)
    LG_TRY(lg::launch_set_jobs(table, k, dj.data() + k,
                               std::min(lg::kJobsPerLaunch, P.njobs - k), st),
           "set jobs");
  LG_TRY(lg::launch_init(table, P.njobs, st), "init");
  if (P.lc.proposer)
    LG_TRY(lg::launch_prop_prep(P.lc.proposer,
                                reinterpret_cast<lg::PropDev*>(ws + P.prop_off), table,
                                P.njobs, st),
           "proposer prep");
  LG_TRY(lg::launch_setup_schedule(table, P.njobs, sc, st), "setup schedule");
  LG_TRY(lg::launch_ingest(table, P.njobs, sc, setup_total(P, lg::kSIngest), st), "ingest");
  const int cols = setup_total(P, lg::kSCols);
  LG_TRY(lg::launch_moments(table, P.njobs, sc, cols, st), "moments");
  if (pf && pf->tm.on) pf->g0 = pf->tm.take(st);
  LG_TRY(lg::launch_gram(table, P.njobs, sc, setup_total(P, lg::kSGram), st), "gram");
  if (pf && pf->tm.on) pf->g1 = pf->tm.take(st);
  if (pf)
    for (int k = 0; k < P.njobs; ++k)
      pf->gram_flops += 2.0 * (double)P.L[k].n * (double)P.L[k].d * (double)P.L[k].d;
  LG_TRY(after_gram(), "after gram");
  LG_TRY(lg::launch_standardize(table, P.njobs, sc, cols, st), "standardize");
  return LINGAM_OK;
}

// Enqueue every step of every job.
int enqueue_steps(const Plan& P, const std::vector<HostJob>& jobs, char* ws, hipStream_t st,
                  lg::Tune tu, Prof* pf, bool ties) {
  lg::JobDev* table = reinterpret_cast<lg::JobDev*>(ws + P.table_off);
  const lg::SchedDev sc = lg::sched_at(ws + P.sched_off, P.njobs);
  // bounded grids: one workgroup of w waves per resident slot
  auto resident = [&](int w) { return P.cu * (lg::kPairWavesPerCu / w); };
  for (int t = 0; t + 1 < P.max_d; ++t) {
    const StepTotals T = step_totals(jobs, P, t, tu, ties);
    if (T.g[lg::kKSel] == 0) break;  // every job finished
    LG_TRY(lg::launch_step_schedule(table, P.njobs, t, P.cu, tu, sc, st), "step schedule");
    if (T.g[lg::kKFeat] > 0 || T.g[lg::kKMlp] > 0)
      LG_TRY(lg::launch_learned_front(table, P.njobs, t, sc, T.g, st), "features / scores");
    if (T.g[lg::kKPairC] > 0) {
      if (pf && pf->tm.on) pf->cand_ev.push_back(pf->tm.take(st));
      LG_TRY(lg::launch_pair_cand(table, P.njobs, sc, T.g[lg::kKPairC], tu.w_rows, st),
             "pair cand");
      if (pf && pf->tm.on) pf->cand_ev.push_back(pf->tm.take(st));
      if (pf) pf->cand_evals += T.cand_evals;
    }
    // learned steps: the full-step kernels are gated on the device, so their
    // host grids are only bounds; bounded grids walk the items instead
    const bool gated = T.g[lg::kKLsel] > 0;
    auto capped = [&](int32_t g, int per_cu) {
      return gated ? std::min<int32_t>(g, P.cu * per_cu) : g;
    };
    if (gated) {
      LG_TRY(lg::launch_learned_back(table, P.njobs, t, sc, T.g, st), "learned decision");
      if (P.lc.extension > 0)
        LG_TRY(lg::launch_susp_schedule(table, P.njobs, sc, 0, P.cu, tu, st),
               "extension schedule");
      if (T.g[lg::kKPairE] > 0) {
        if (pf && pf->tm.on) pf->cand_ev.push_back(pf->tm.take(st));
        LG_TRY(lg::launch_pair_ext(table, P.njobs, sc,
                                   std::min<int32_t>(T.g[lg::kKPairE], resident(tu.w_rows)),
                                   tu.w_rows, st),
               "pair ext");
        if (pf && pf->tm.on) pf->cand_ev.push_back(pf->tm.take(st));
        LG_TRY(lg::launch_ext_back(table, P.njobs, t, sc,
                                   std::min<int32_t>(T.g[lg::kKBoundE], P.cu * 4),
                                   std::min<int32_t>(T.g[lg::kKCompE], P.njobs), st),
               "extension bounds");
      }
      LG_TRY(lg::launch_susp_schedule(table, P.njobs, sc, 1, P.cu, tu, st),
             "suspect schedule");
      if (T.g[lg::kKPairS] > 0) {
        if (pf && pf->tm.on) pf->cand_ev.push_back(pf->tm.take(st));
        LG_TRY(lg::launch_pair_susp(table, P.njobs, sc,
                                    std::min<int32_t>(T.g[lg::kKPairS], resident(tu.w_rows)),
                                    tu.w_rows, st),
               "pair susp");
        if (pf && pf->tm.on) pf->cand_ev.push_back(pf->tm.take(st));
      }
      LG_TRY(lg::launch_susp_back(table, P.njobs, t, sc,
                                  std::min<int32_t>(T.g[lg::kKCombS], P.cu * 8),
                                  std::min<int32_t>(T.g[lg::kKRowkS], P.cu * 4),
                                  std::min<int32_t>(T.g[lg::kKLsel2], P.njobs), st),
             "suspect decision");
      LG_TRY(lg::launch_gate_schedule(table, P.njobs, sc, st), "gate schedule");
    }
    if (T.g[lg::kKPair] > 0) {
      if (pf && pf->tm.on) pf->pair_ev.push_back(pf->tm.take(st));
      LG_TRY(lg::launch_pair(table, P.njobs, sc,
                             gated ? std::min<int32_t>(T.g[lg::kKPair], resident(tu.w_all))
                                   : T.g[lg::kKPair],
                             tu.w_all, st, gated),
             "pair");
      if (pf && pf->tm.on) pf->pair_ev.push_back(pf->tm.take(st));
      if (pf) pf->pair_evals += T.pair_evals;
      LG_TRY(lg::launch_combine(table, P.njobs, sc, capped(T.g[lg::kKComb], 8), st),
             "combine");
    }
    LG_TRY(lg::launch_pair64(table, P.njobs, sc, T.g[lg::kKP64], st), "pair64");
    LG_TRY(lg::launch_rowk(table, P.njobs, sc, capped(T.g[lg::kKRowk], 8), st), "rowk");
    LG_TRY(lg::launch_select(table, P.njobs, t, sc, T.g[lg::kKSel], st), "select");
    // near-ties of FP32-path steps (full or learned) decided in FP64
    if (ties && (T.g[lg::kKPair] > 0 || gated))
      LG_TRY(lg::launch_tie(table, P.njobs, sc, t, P.cu, st), "tie");
    if (T.g[lg::kKRes] > 0) {
      if (pf && pf->tm.on) pf->resid_ev.push_back(pf->tm.take(st));
      LG_TRY(lg::launch_resid(table, P.njobs, sc, T.g[lg::kKRes], st), "resid");
      if (pf && pf->tm.on) pf->resid_ev.push_back(pf->tm.take(st));
      if (pf) pf->resid_bytes += T.resid_bytes;
    }
  }
  return LINGAM_OK;
}

// --------------------------------------------------------------------------
// launch-shape autotuner
// --------------------------------------------------------------------------

const lg::Tune kDefaultTune{16, 8, 4, 4};
// split policies (target workgroups per CU, least sample iterations per split)
const int32_t kSplitCandidates[][2] = {{8, 8}, {16, 8}, {16, 4}, {32, 4}, {8, 16}, {16, 16}};
const int32_t kWaveChoices[] = {4, 2, 1};

int ilog2_ceil(double x) {
  int k = 0;
  while ((double)(1LL << k) < x && k < 62) ++k;
  return k;
}

// Bucket key: total sample-pair work, largest padded n, number of jobs, and
// the candidate cap of the learned form (0: plain).
std::string tune_key(const std::vector<HostJob>& jobs, const Plan& P) {
  double work = 0.0;
  int64_t maxn = 0;
  for (int k = 0; k < P.njobs; ++k) {
    work += (double)jobs[k].n * ((double)jobs[k].d * jobs[k].d * jobs[k].d) / 3.0;
    maxn = std::max<int64_t>(maxn, P.L[k].n_pad);
  }
  char buf[112];
  snprintf(buf, sizeof(buf), "gfx950/cu%d/w%d/n%d/j%d/k%d", P.cu, ilog2_ceil(work),
           ilog2_ceil((double)maxn), ilog2_ceil((double)P.njobs),
           P.lc.proposer ? P.lc.K : 0);
  return buf;
}

bool valid_tune(const lg::Tune& t) {
  return t.target_per_cu >= 1 && t.target_per_cu <= lg::kMaxTargetPerCu &&
         t.min_iters >= lg::kMinMinIters && lg::valid_waves(t.w_all) &&
         lg::valid_waves(t.w_rows);
}

// Persistent cache: one "key target min_iters w_all w_rows" line per entry in
// the file named by LINGAM_AUTOTUNE_CACHE (when that variable is set).
void load_tune_file(DevState& ds) {
  if (ds.tunes_loaded) return;
  ds.tunes_loaded = true;
  const char* path = getenv("LINGAM_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[128];
  lg::Tune t{};
  while (fscanf(f, "%127s %d %d %d %d", key, &t.target_per_cu, &t.min_iters, &t.w_all,
                &t.w_rows) == 5)
    if (valid_tune(t)) ds.tunes[key] = t;
  fclose(f);
}

void save_tune_file(const DevState& ds) {
  const char* path = getenv("LINGAM_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  for (const auto& kv : ds.tunes)
    fprintf(f, "%s %d %d %d %d\n", kv.first.c_str(), kv.second.target_per_cu,
            kv.second.min_iters, kv.second.w_all, kv.second.w_rows);
  fclose(f);
}

// Time the pair kernels of a few sampled steps on the call's own data (after
// the set-up; the pair kernels only write their partial-sum scratch, and
// every position below m is valid while the active list is still the
// identity), in three rounds: the split policy (the only choice that moves
// results, at the rounding level), then the waves per workgroup of the
// all-pairs kernel, then, for the learned form, of the row kernels.  Row
// kernels are timed on the candidate pass after that step's features, scores
// and top-K; the learned form's split policy is timed there too, since its
// candidate passes, not the all-pairs kernel, carry its pair work.  Ties keep
// the earlier candidate.
int autotune(const Plan& P, const std::vector<HostJob>& jobs, char* ws, hipStream_t st,
             bool ties, lg::Tune* out) {
  lg::JobDev* table = reinterpret_cast<lg::JobDev*>(ws + P.table_off);
  const lg::SchedDev sc = lg::sched_at(ws + P.sched_off, P.njobs);
  std::vector<int> steps;
  const int dmax = P.max_d;
  for (double f : {0.0, 0.25, 0.5, 0.7, 0.85}) {
    const int t = (int)(f * dmax);
    if (dmax - t > lg::kFp64MaxM) steps.push_back(t);
  }
  *out = kDefaultTune;
  if (steps.empty()) return LINGAM_OK;
  const bool learned = P.lc.proposer != nullptr;
  Timer tm;
  // summed time of the sampled steps' pair kernel (all pairs, or candidate rows)
  auto time_steps = [&](const lg::Tune& c, bool rows, double* total) -> int {
    std::vector<std::pair<int, int>> ev;
    for (int t : steps) {
      const StepTotals T = step_totals(jobs, P, t, c, ties);
      const int kind = rows ? lg::kKPairC : lg::kKPair;
      if (T.g[kind] <= 0) continue;
      LG_TRY(lg::launch_step_schedule(table, P.njobs, t, P.cu, c, sc, st), "tune schedule");
      if (rows)
        LG_TRY(lg::launch_learned_front(table, P.njobs, t, sc, T.g, st), "tune front");
      const int a = tm.take(st);
      if (rows)
        LG_TRY(lg::launch_pair_cand(table, P.njobs, sc, T.g[kind], c.w_rows, st), "tune cand");
      else
        LG_TRY(lg::launch_pair(table, P.njobs, sc, T.g[kind], c.w_all, st), "tune pair");
      ev.emplace_back(a, tm.take(st));
    }
    LG_TRY(hipStreamSynchronize(st), "tune sync");
    *total = 0.0;
    for (auto& e : ev) *total += tm.ms(e.first, e.second);
    if (ev.empty()) *total = -1.0;
    return LINGAM_OK;
  };
  // every candidate is timed in two rounds (candidates in turn, so a drift
  // in clocks touches them alike) and scored by its faster round
  auto pick = [&](lg::Tune c, int field, const int32_t* vals, int nv) -> int {
    auto set = [&](int i) {
      if (field == 0) {
        c.target_per_cu = vals[2 * i];
        c.min_iters = vals[2 * i + 1];
      } else if (field == 1) {
        c.w_all = vals[i];
      } else {
        c.w_rows = vals[i];
      }
      return c;
    };
    std::vector<double> score(nv, -1.0);
    for (int round = 0; round < 2; ++round)
      for (int i = 0; i < nv; ++i) {
        double ms = 0.0;
        const int rc = time_steps(set(i), field == 2 || (field == 0 && learned), &ms);
        if (rc != LINGAM_OK) return rc;
        if (ms >= 0.0 && (score[i] < 0.0 || ms < score[i])) score[i] = ms;
      }
    double best = 1e300;
    for (int i = 0; i < nv; ++i)
      if (score[i] >= 0.0 && score[i] < best) {
        best = score[i];
        *out = set(i);
      }
    return LINGAM_OK;
  };
  int rc = pick(kDefaultTune, 0, &kSplitCandidates[0][0],
                (int)(sizeof(kSplitCandidates) / sizeof(kSplitCandidates[0])));
  if (rc == LINGAM_OK) rc = pick(*out, 1, kWaveChoices, 3);
  if (rc == LINGAM_OK && learned) rc = pick(*out, 2, kWaveChoices, 3);
  return rc;
}

// --------------------------------------------------------------------------
// one call of the engine
// --------------------------------------------------------------------------

// Everything a captured call bakes into its kernels' arguments: the device
// job records (data, outputs and workspace regions), the workspace, the split
// policy, the CU count, and the learned-form configuration (the caller's
// proposer buffer is read by the captured network copy).
std::string graph_key(const std::vector<lg::JobDev>& dj, const Plan& P, void* ws, lg::Tune tu) {
  std::string k;
  k.append(reinterpret_cast<const char*>(dj.data()), dj.size() * sizeof(lg::JobDev));
  char buf[256];
  snprintf(buf, sizeof(buf), "|%p|%zu|%d|%d|%d|%d|%d|%p|%d|%d|%d|%d|%d|%a", ws, P.total,
           tu.target_per_cu, tu.min_iters, tu.w_all, tu.w_rows, P.cu,
           (const void*)P.lc.proposer, P.lc.K,
           P.lc.min_m, P.lc.audit_every, P.lc.max_suspects, P.lc.extension, (double)P.lc.delta);
  k.append(buf);
  return k;
}

int finish(const Plan& P, const std::vector<lg::JobDev>& dj, char* ws, const lingam_opts* opts,
           int32_t* job_status, hipStream_t st, Prof& pf) {
  if (job_status)
    LG_TRY(lg::launch_gather_status(reinterpret_cast<lg::JobDev*>(ws + P.table_off), P.njobs,
                                    job_status, st),
           "gather status");
  if (opts->dev_status)
    LG_TRY(hipMemcpyAsync(opts->dev_status, dj[0].ctrl, sizeof(int32_t),
                          hipMemcpyDeviceToDevice, st),
           "status copy");
  if (pf.tm.on) pf.all1 = pf.tm.take(st);
  const bool sync = !(opts->flags & LINGAM_FLAG_NO_SYNC) || pf.tm.on;
  if (!sync) return LINGAM_OK;
  std::vector<lg::Ctrl> ctrl(P.njobs);
  for (int k = 0; k < P.njobs; ++k)
    LG_TRY(hipMemcpyAsync(&ctrl[k], dj[k].ctrl, sizeof(lg::Ctrl), hipMemcpyDeviceToHost, st),
           "hipMemcpyAsync(control)");
  // learned steps whose full search was gated off (for the profile's counts)
  std::vector<std::vector<int32_t>> logs;
  if (P.lc.proposer && pf.tm.on && opts->profile) {
    logs.resize(P.njobs);
    for (int k = 0; k < P.njobs; ++k) {
      logs[k].resize((size_t)P.L[k].d);
      LG_TRY(hipMemcpyAsync(logs[k].data(), dj[k].steplog, sizeof(int32_t) * logs[k].size(),
                            hipMemcpyDeviceToHost, st),
             "hipMemcpyAsync(step log)");
    }
  }
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  std::vector<int32_t> st_host(P.njobs, 0);
  for (int k = 0; k < P.njobs; ++k) st_host[k] = ctrl[k].status;
  if (P.lc.proposer && opts->learned_stats) {
    lingam_learned_stats* ls = opts->learned_stats;
    memset(ls, 0, sizeof(*ls));
    for (const lg::Ctrl& c : ctrl) {
      ls->learned_steps += c.n_learned;
      ls->certified += c.n_certified;
      ls->fallbacks += c.n_fallback;
      ls->audits += c.n_audit;
      ls->audit_agree += c.n_audit_agree;
      ls->suspects_max = std::max(ls->suspects_max, c.n_suspects_max);
      ls->suspects_sum += c.n_suspects_sum;
      ls->expanded += c.n_expanded;
      ls->cleared += c.n_cleared;
      ls->rows_sum += c.n_rows_sum;
    }
  }
  if (pf.tm.on && opts->profile) {
    lingam_profile* pr = opts->profile;
    memset(pr, 0, sizeof(*pr));
    pr->total_ms = pf.tm.ms(pf.all0, pf.all1);
    pr->gram_ms = pf.tm.ms(pf.g0, pf.g1);
    pr->gram_flops = pf.gram_flops;
    for (size_t k = 0; k + 1 < pf.pair_ev.size(); k += 2)
      pr->pair_ms += pf.tm.ms(pf.pair_ev[k], pf.pair_ev[k + 1]);
    pr->pair_launches = (int64_t)(pf.pair_ev.size() / 2);
    pr->pair_evals = pf.pair_evals;
    for (size_t k = 0; k + 1 < pf.resid_ev.size(); k += 2)
      pr->resid_ms += pf.tm.ms(pf.resid_ev[k], pf.resid_ev[k + 1]);
    pr->resid_bytes = pf.resid_bytes;
    for (size_t k = 0; k + 1 < pf.cand_ev.size(); k += 2)
      pr->cand_ms += pf.tm.ms(pf.cand_ev[k], pf.cand_ev[k + 1]);
    pr->cand_launches = (int64_t)(pf.cand_ev.size() / 2);
    pr->cand_evals = pf.cand_evals;
    for (const lg::Ctrl& c : ctrl) {
      pr->tie_steps += c.n_ties;
      pr->tie_rows += c.n_tie_rows;
      pr->tie_overflow += c.n_tie_overflow;
    }
    // steps a learned decision took did not run the all-pairs kernel; steps
    // decided by the second pass measured their suspects against the
    // extension columns, then the remaining suspects' rows
    for (int k = 0; k < (int)logs.size(); ++k) {
      const int64_t d = P.L[k].d, n = P.L[k].n;
      for (int64_t t = 0; t + 1 < d; ++t) {
        const int64_t m = d - t;
        const int32_t e = logs[k][(size_t)t];
        const int32_t kind = e & 15, nsus = (e >> 4) & 0xFFF, rows = e >> 16;
        if ((kind == 1 || kind == 4) && m > lg::kFp64MaxM)
          pr->pair_evals -= (double)m * (double)(m - 1) * (double)n;
        if (kind == 4) {
          const int32_t ne =
              lg::ext_count((int32_t)m, lg::step_topk((int32_t)m, P.lc.K), P.lc.extension);
          pr->cand_evals += 2.0 * nsus * (double)ne * (double)n;
          pr->cand_evals += 2.0 * rows * (double)(m - 1) * (double)n;
        }
      }
    }
  }
  for (int k = 0; k < P.njobs; ++k)
    if (st_host[k] != 0) return status_from_device(st_host[k]);
  return LINGAM_OK;
}

// Run a batch: (autotune), set-up, steps, status.  `fill` writes the data rows
// of jobs that have no X (VarLiNGAM residuals); `after_gram` and `after` hook
// into the set-up and the end.
template <typename Fill, typename AfterGram, typename After>
int run_engine(const Plan& P, const std::vector<HostJob>& jobs, const lingam_opts* opts,
               int32_t* job_status, char* ws, hipStream_t st, Fill fill, AfterGram after_gram,
               After after) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc != LINGAM_OK) return rc;
  const bool ties = !(opts->flags & LINGAM_FLAG_FP32_TIES);
  const std::vector<lg::JobDev> dj = device_jobs(P, jobs, ws, ties);
  Prof pf;
  pf.tm.on = opts->profile != nullptr;

  // split policy: cached result, or tune now when asked
  lg::Tune tu = kDefaultTune;
  const std::string tkey = tune_key(jobs, P);
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_tune_file(g_dev[dev]);
    auto it = g_dev[dev].tunes.find(tkey);
    if (it != g_dev[dev].tunes.end()) {
      tu = it->second;
      have = true;
    }
  }
  if ((opts->flags & LINGAM_FLAG_AUTOTUNE) && !have) {
    rc = fill();
    if (rc != LINGAM_OK) return rc;
    rc = enqueue_setup(P, dj, ws, st, nullptr, [] { return hipSuccess; });
    if (rc != LINGAM_OK) return rc;
    rc = autotune(P, jobs, ws, st, ties, &tu);
    if (rc != LINGAM_OK) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    g_dev[dev].tunes[tkey] = tu;
    save_tune_file(g_dev[dev]);
  }

  // a launch shape the caller fixed (the results do not depend on it)
  if (opts->waves_all) tu.w_all = opts->waves_all;
  if (opts->waves_rows) tu.w_rows = opts->waves_rows;

  const bool graph = (opts->flags & LINGAM_FLAG_GRAPH) && !pf.tm.on;
  if (pf.tm.on) pf.all0 = pf.tm.take(st);
  if (!graph) {
    rc = fill();
    if (rc != LINGAM_OK) return rc;
    rc = enqueue_setup(P, dj, ws, st, &pf, after_gram);
    if (rc != LINGAM_OK) return rc;
    rc = enqueue_steps(P, jobs, ws, st, tu, &pf, ties);
    if (rc != LINGAM_OK) return rc;
    rc = after();
    if (rc != LINGAM_OK) return rc;
    return finish(P, dj, ws, opts, job_status, st, pf);
  }

  // graph mode: capture the whole call once per (jobs, workspace, policy) and
  // replay the instantiated graph on later identical calls
  const std::string gkey = graph_key(dj, P, ws, tu);
  hipGraphExec_t exec = nullptr;
  std::lock_guard<std::mutex> lk(g_mu);  // one capture / cache update at a time
  DevState& ds = g_dev[dev];
  for (auto it = ds.graphs.begin(); it != ds.graphs.end(); ++it)
    if (it->key == gkey) {
      exec = it->exec;
      ds.graphs.splice(ds.graphs.begin(), ds.graphs, it);
      break;
    }
  if (!exec) {
    if (!ds.capture) LG_TRY(hipStreamCreateWithFlags(&ds.capture, hipStreamNonBlocking), "stream");
    hipStream_t cap = ds.capture;
    LG_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
    int rc2 = fill();
    if (rc2 == LINGAM_OK) rc2 = enqueue_setup(P, dj, ws, cap, nullptr, after_gram);
    if (rc2 == LINGAM_OK) rc2 = enqueue_steps(P, jobs, ws, cap, tu, nullptr, ties);
    if (rc2 == LINGAM_OK) rc2 = after();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g);
    if (rc2 != LINGAM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc2;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate");
    ds.graphs.push_front(GraphEntry{gkey, exec});
    while (ds.graphs.size() > 8) {
      (void)hipGraphExecDestroy(ds.graphs.back().exec);
      ds.graphs.pop_back();
    }
  }
  LG_TRY(hipGraphLaunch(exec, st), "hipGraphLaunch");
  return finish(P, dj, ws, opts, job_status, st, pf);
}

int check_learn(const lingam_opts* opts) {
  if ((opts->waves_all && !lg::valid_waves(opts->waves_all)) ||
      (opts->waves_rows && !lg::valid_waves(opts->waves_rows)))
    return fail(LINGAM_E_INVALID, "waves_all %d / waves_rows %d must be 0, 1, 2 or 4",
                opts->waves_all, opts->waves_rows);
  if (!opts->proposer) return LINGAM_OK;
  if (opts->topk < 8 || opts->topk > lg::kMaxTopK || opts->topk % 8 != 0)
    return fail(LINGAM_E_INVALID, "topk %d must be a multiple of 8 in [8, %d]", opts->topk,
                lg::kMaxTopK);
  if (opts->audit_every < 0)
    return fail(LINGAM_E_INVALID, "audit_every %d < 0", opts->audit_every);
  const int32_t k_lo = opts->topk < 64 ? opts->topk : 64;
  if (opts->learned_min_m < 2 * k_lo || opts->learned_min_m < lg::kFp64MaxM)
    return fail(LINGAM_E_INVALID, "learned_min_m %d must be >= 2 min(topk, 64) and >= %d",
                opts->learned_min_m, lg::kFp64MaxM);
  if (opts->margin != opts->margin) return fail(LINGAM_E_INVALID, "margin is NaN");
  if (opts->max_suspects < 0)
    return fail(LINGAM_E_INVALID, "max_suspects %d < 0", opts->max_suspects);
  if (opts->extension < 0 || opts->extension > lg::kMaxExt || opts->extension % 8 != 0)
    return fail(LINGAM_E_INVALID, "extension %d must be a multiple of 8 in [0, %d]",
                opts->extension, lg::kMaxExt);
  return LINGAM_OK;
}

int check_opts(const lingam_opts* opts, int64_t d) {
  if (opts->struct_size != sizeof(lingam_opts))
    return fail(LINGAM_E_INVALID, "opts->struct_size %u != %zu", opts->struct_size,
                sizeof(lingam_opts));
  const int rc = check_learn(opts);
  if (rc != LINGAM_OK) return rc;
  if (opts->forced_len < 0 || opts->forced_len > d)
    return fail(LINGAM_E_INVALID, "forced_len %d outside [0, d]", opts->forced_len);
  if (opts->forced_len > 0 && !opts->forced_order)
    return fail(LINGAM_E_INVALID, "forced_len > 0 but forced_order is NULL");
  return LINGAM_OK;
}

int check_job(const HostJob& j, int k) {
  if (!j.X || !j.order) return fail(LINGAM_E_INVALID, "job %d: X and order must be non-NULL", k);
  if (j.n < 2)
    return fail(LINGAM_E_INVALID, "job %d: need n >= 2 samples (got %lld)", k, (long long)j.n);
  if (j.d < 1)
    return fail(LINGAM_E_INVALID, "job %d: need d >= 1 variables (got %lld)", k, (long long)j.d);
  if (j.ldx < j.d)
    return fail(LINGAM_E_INVALID, "job %d: ldx (%lld) < d (%lld)", k, (long long)j.ldx,
                (long long)j.d);
  if (!j.rows && j.n_src < j.n)
    return fail(LINGAM_E_INVALID, "job %d: n (%lld) > rows of X (%lld)", k, (long long)j.n,
                (long long)j.n_src);
  if (j.n_src < 1) return fail(LINGAM_E_INVALID, "job %d: X has no rows", k);
  if (j.n > kMaxN || j.d > kMaxD || j.n_src > kMaxN)
    return fail(LINGAM_E_UNSUPPORTED, "job %d: n <= %lld and d <= %lld supported", k,
                (long long)kMaxN, (long long)kMaxD);
  return LINGAM_OK;
}

int ok_fill() { return LINGAM_OK; }
hipError_t ok_hip() { return hipSuccess; }

}  // namespace

extern "C" {

void lingam_opts_init(lingam_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(lingam_opts);
  o->topk = 64;
  o->audit_every = 0;
  o->margin = INFINITY;
  o->learned_min_m = 128;
  o->max_suspects = lg::kMaxSuspects;
  o->extension = 0;
}

const char* lingam_last_error(void) { return g_err; }

const char* lingam_version(void) { return "lingam-mi355x 0.2 (gfx950)"; }

size_t lingam_workspace_size(int64_t n, int64_t d, const lingam_opts* opts) {
  if (n < 2 || d < 1 || n > kMaxN || d > kMaxD) return 0;
  if (opts && (opts->struct_size != sizeof(lingam_opts) || check_learn(opts) != LINGAM_OK))
    return 0;
  int cu = 0;
  if (num_cu_of_current(&cu) != LINGAM_OK) cu = 256;
  HostJob j{};
  j.n = n;
  j.d = d;
  return make_plan({j}, cu, learn_of(opts)).total;
}

}  // extern "C"

namespace {

// lingam_causal_order with the workspace given (ws) or, when noalloc, the
// current device's scratch array.
int causal_order_impl(const float* X, int64_t n, int64_t d, int64_t ldx, int32_t* order,
                      const lingam_opts* opts, void* ws, size_t ws_bytes, void* stream,
                      bool noalloc) {
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
  if (ldx < d)
    return fail(LINGAM_E_INVALID, "ldx (%lld) < d (%lld)", (long long)ldx, (long long)d);
  if (n > kMaxN || d > kMaxD)
    return fail(LINGAM_E_UNSUPPORTED, "n <= %lld and d <= %lld supported", (long long)kMaxN,
                (long long)kMaxD);
  int rc = check_opts(opts, d);
  if (rc != LINGAM_OK) return rc;
  if (noalloc && (opts->flags & (LINGAM_FLAG_GRAPH | LINGAM_FLAG_AUTOTUNE)))
    return fail(LINGAM_E_UNSUPPORTED,
                "lingam_causal_order_noalloc: LINGAM_FLAG_GRAPH and LINGAM_FLAG_AUTOTUNE are "
                "not available (graph instantiation and tuning allocate)");
  if (noalloc && opts->profile)
    return fail(LINGAM_E_UNSUPPORTED, "lingam_causal_order_noalloc: no profile");
  int cu = 0;
  rc = num_cu_of_current(&cu);
  if (rc != LINGAM_OK) return rc;
  const HostJob j{X,     nullptr, n, ldx, n, d, order, opts->step_measures, opts->step_gap,
                  opts->forced_order, opts->forced_len, opts->record_features, opts->step_log};
  const std::vector<HostJob> jobs{j};
  const Plan P = make_plan(jobs, cu, learn_of(opts));
  if (noalloc) {
    if (P.total > (size_t)LINGAM_NOALLOC_SCRATCH_BYTES)
      return fail(LINGAM_E_UNSUPPORTED,
                  "lingam_causal_order_noalloc: n=%lld d=%lld needs %zu bytes of workspace, "
                  "the scratch array holds %zu",
                  (long long)n, (long long)d, P.total, (size_t)LINGAM_NOALLOC_SCRATCH_BYTES);
    int dev = 0;
    rc = current_device(&dev);
    if (rc != LINGAM_OK) return rc;
    LG_TRY(lg::noalloc_scratch(dev, &ws), "hipGetSymbolAddress(scratch)");
    ws_bytes = (size_t)LINGAM_NOALLOC_SCRATCH_BYTES;
  }
  if (!ws || ws_bytes < P.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", P.total,
                ws ? ws_bytes : (size_t)0);
  return run_engine(P, jobs, opts, nullptr, (char*)ws, (hipStream_t)stream, ok_fill, ok_hip,
                    ok_fill);
}

}  // namespace

extern "C" {

int lingam_causal_order(const float* X, int64_t n, int64_t d, int64_t ldx, int32_t* order,
                        const lingam_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  return causal_order_impl(X, n, d, ldx, order, opts, ws, ws_bytes, stream, false);
}

int lingam_causal_order_noalloc(const float* X, int64_t n, int64_t d, int64_t ldx,
                                int32_t* order, const lingam_opts* opts, void* stream) {
  return causal_order_impl(X, n, d, ldx, order, opts, nullptr, 0, stream, true);
}

static int batch_jobs(const lingam_job* jobs, int32_t n_jobs, std::vector<HostJob>* out) {
  if (!jobs || n_jobs < 1) return fail(LINGAM_E_INVALID, "need at least one job");
  if (n_jobs > kMaxJobs) return fail(LINGAM_E_UNSUPPORTED, "at most %d jobs", kMaxJobs);
  out->clear();
  for (int k = 0; k < n_jobs; ++k) {
    const lingam_job& s = jobs[k];
    const HostJob h{s.X,        s.rows, s.n_rows, s.ldx, s.n, s.d, s.order, s.step_measures,
                    s.step_gap, nullptr, 0,      s.record_features};
    const int rc = check_job(h, k);
    if (rc != LINGAM_OK) return rc;
    out->push_back(h);
  }
  return LINGAM_OK;
}

size_t lingam_batch_workspace_size(const lingam_job* jobs, int32_t n_jobs,
                                   const lingam_opts* opts) {
  if (opts && (opts->struct_size != sizeof(lingam_opts) || check_learn(opts) != LINGAM_OK))
    return 0;
  if (opts && opts->proposer && opts->extension > 0) return 0;
  std::vector<HostJob> hj;
  if (batch_jobs(jobs, n_jobs, &hj) != LINGAM_OK) return 0;
  int cu = 0;
  if (num_cu_of_current(&cu) != LINGAM_OK) cu = 256;
  return make_plan(hj, cu, learn_of(opts)).total;
}

int lingam_batch_causal_order(const lingam_job* jobs, int32_t n_jobs, int32_t* job_status,
                              const lingam_opts* opts, void* ws, size_t ws_bytes,
                              void* stream) {
  g_err[0] = 0;
  lingam_opts dflt;
  lingam_opts_init(&dflt);
  if (!opts) opts = &dflt;
  if (opts->struct_size != sizeof(lingam_opts))
    return fail(LINGAM_E_INVALID, "opts->struct_size %u != %zu", opts->struct_size,
                sizeof(lingam_opts));
  if (opts->forced_len != 0 || opts->step_measures || opts->step_gap || opts->dev_status)
    return fail(LINGAM_E_INVALID,
                "batched calls take per-step outputs in lingam_job, status in job_status, and "
                "no forcing");
  int rc = check_learn(opts);
  if (rc != LINGAM_OK) return rc;
  if (opts->proposer && opts->extension > 0)
    return fail(LINGAM_E_UNSUPPORTED, "extension columns are available to single orderings only");
  std::vector<HostJob> hj;
  rc = batch_jobs(jobs, n_jobs, &hj);
  if (rc != LINGAM_OK) return rc;
  int cu = 0;
  rc = num_cu_of_current(&cu);
  if (rc != LINGAM_OK) return rc;
  const Plan P = make_plan(hj, cu, learn_of(opts));
  if (!ws || ws_bytes < P.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", P.total,
                ws ? ws_bytes : (size_t)0);
  return run_engine(P, hj, opts, job_status, (char*)ws, (hipStream_t)stream, ok_fill, ok_hip,
                    ok_fill);
}

size_t varlingam_workspace_size(int64_t T, int64_t d, int32_t lags, const lingam_opts* opts) {
  if (d < 1 || lags < 1 || d > kMaxD || T > kMaxN) return 0;
  if (opts && (opts->struct_size != sizeof(lingam_opts) || check_learn(opts) != LINGAM_OK))
    return 0;
  if (T - lags < 1 + (int64_t)lags * d + 1) return 0;
  int cu = 0;
  if (num_cu_of_current(&cu) != LINGAM_OK) cu = 256;
  HostJob j{};
  j.n = T - lags;
  j.d = d;
  const Plan P = make_plan({j}, cu, learn_of(opts));
  return align256(P.total) + lg::make_var_layout(T, d, lags, cu).total;
}

int varlingam_fit(const float* X, int64_t T, int64_t d, int64_t ldx, int32_t lags, double* M,
                  float* resid, int32_t* order, double* B0, const lingam_opts* opts, void* ws,
                  size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  lingam_opts dflt;
  lingam_opts_init(&dflt);
  if (!opts) opts = &dflt;
  if (opts->struct_size != sizeof(lingam_opts))
    return fail(LINGAM_E_INVALID, "opts->struct_size %u != %zu", opts->struct_size,
                sizeof(lingam_opts));
  if (!X || !order) return fail(LINGAM_E_INVALID, "X and order must be non-NULL");
  if (d < 1) return fail(LINGAM_E_INVALID, "need d >= 1 variables (got %lld)", (long long)d);
  if (ldx < d)
    return fail(LINGAM_E_INVALID, "ldx (%lld) < d (%lld)", (long long)ldx, (long long)d);
  if (lags < 1) return fail(LINGAM_E_INVALID, "need lags >= 1 (got %d)", lags);
  if (d > kMaxD || T > kMaxN || (int64_t)lags * d + 1 > 8192)
    return fail(LINGAM_E_UNSUPPORTED, "d <= %lld, T <= %lld and lags * d < 8192 supported",
                (long long)kMaxD, (long long)kMaxN);
  if (T - lags < 1 + (int64_t)lags * d + 1)
    return fail(LINGAM_E_INVALID, "T - lags (%lld) must exceed the %lld regressors",
                (long long)(T - lags), (long long)(1 + (int64_t)lags * d));
  int rc = check_opts(opts, d);
  if (rc != LINGAM_OK) return rc;
  if (opts->flags & LINGAM_FLAG_GRAPH)
    return fail(LINGAM_E_UNSUPPORTED, "varlingam_fit does not take LINGAM_FLAG_GRAPH");
  int cu = 0;
  rc = num_cu_of_current(&cu);
  if (rc != LINGAM_OK) return rc;
  // the VAR residuals are the job's data rows: no X for the ingest kernel
  const HostJob j{nullptr,         nullptr,      T - lags, d, T - lags, d, order,
                  opts->step_measures, opts->step_gap, opts->forced_order, opts->forced_len,
                  opts->record_features, opts->step_log};
  const std::vector<HostJob> jobs{j};
  const Plan P = make_plan(jobs, cu, learn_of(opts));
  const lg::VarLayout V = lg::make_var_layout(T, d, lags, cu);
  const size_t var_off = align256(P.total);
  if (!ws || ws_bytes < var_off + V.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)",
                var_off + V.total, ws ? ws_bytes : (size_t)0);
  char* w = (char*)ws;
  char* vw = w + var_off;
  char* job = w + P.job_off[0];
  hipStream_t st = (hipStream_t)stream;
  return run_engine(
      P, jobs, opts, nullptr, w, st,
      [&]() -> int {
        LG_TRY(lg::launch_var_fit(V, vw, job, X, ldx, resid, M, st), "var fit");
        return LINGAM_OK;
      },
      [&] { return B0 ? lg::launch_save_rho(V, vw, job, st) : hipSuccess; },
      [&]() -> int {
        if (B0) LG_TRY(lg::launch_b0(V, vw, job, order, B0, st), "b0");
        return LINGAM_OK;
      });
}

size_t lingam_adjacency_workspace_size(int64_t n, int64_t d) {
  if (n < 2 || d < 1 || n > kMaxN || d > kMaxD) return 0;
  return lg::make_adj_layout(n, d).total;
}

int lingam_adjacency(const float* X, int64_t n_rows, int64_t ldx, const int32_t* rows, int64_t n,
                     int64_t d, const int32_t* order, double* B, void* ws, size_t ws_bytes,
                     void* stream) {
  g_err[0] = 0;
  if (!X || !order || !B) return fail(LINGAM_E_INVALID, "X, order and B must be non-NULL");
  if (n < 2 || d < 1 || ldx < d || n_rows < 1 || (!rows && n > n_rows))
    return fail(LINGAM_E_INVALID, "bad sizes n=%lld d=%lld ldx=%lld n_rows=%lld", (long long)n,
                (long long)d, (long long)ldx, (long long)n_rows);
  if (n > kMaxN || d > kMaxD || n_rows > kMaxN)
    return fail(LINGAM_E_UNSUPPORTED, "size beyond supported range");
  const lg::AdjLayout A = lg::make_adj_layout(n, d);
  if (!ws || ws_bytes < A.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", A.total,
                ws ? ws_bytes : (size_t)0);
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  int32_t s = 0;
  // the order and the row map index device arrays: check them before
  // anything reads through them
  LG_TRY(lg::launch_adj_check(A, w, order, rows, n_rows, st), "adjacency check");
  LG_TRY(hipMemcpyAsync(&s, w + A.ctrl, sizeof(int32_t), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync(status)");
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s != 0)
    return fail(LINGAM_E_INVALID,
                "order is not a permutation of 0 .. d-1, or a row index is outside [0, n_rows)");
  LG_TRY(lg::launch_adjacency(A, w, X, ldx, rows, order, B, st), "adjacency launch");
  LG_TRY(hipMemcpyAsync(&s, w + A.ctrl, sizeof(int32_t), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync(status)");
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s != 0)
    return fail(LINGAM_E_DEGENERATE,
                "non-finite data or a covariance that is not positive definite");
  return LINGAM_OK;
}

size_t lingam_adjacency_pruned_workspace_size(int64_t n, int64_t d) {
  if (n < 2 || d < 1 || n > kMaxN || d > kMaxD) return 0;
  return lg::make_prune_layout(n, d).total;
}

int lingam_adjacency_pruned(const float* X, int64_t n_rows, int64_t ldx, const int32_t* rows,
                            int64_t n, int64_t d, const int32_t* order, int32_t max_active,
                            double* B, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!X || !order || !B) return fail(LINGAM_E_INVALID, "X, order and B must be non-NULL");
  if (n < 2 || d < 1 || ldx < d || n_rows < 1 || (!rows && n > n_rows))
    return fail(LINGAM_E_INVALID, "bad sizes n=%lld d=%lld ldx=%lld n_rows=%lld", (long long)n,
                (long long)d, (long long)ldx, (long long)n_rows);
  if (max_active < 1 || max_active > lg::kLassoMaxActive)
    return fail(LINGAM_E_INVALID, "max_active %d outside [1, %d]", max_active,
                lg::kLassoMaxActive);
  if (n > kMaxN || d > kMaxD || n_rows > kMaxN)
    return fail(LINGAM_E_UNSUPPORTED, "size beyond supported range");
  if (n <= d + 1)
    return fail(LINGAM_E_DEGENERATE, "n (%lld) must exceed d + 1 (%lld)", (long long)n,
                (long long)(d + 1));
  const lg::PruneLayout A = lg::make_prune_layout(n, d);
  if (!ws || ws_bytes < A.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", A.total,
                ws ? ws_bytes : (size_t)0);
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  lg::AdjLayout V{};  // the check's view of the same status and mark regions
  V.n = n;
  V.d = d;
  V.ctrl = A.ctrl;
  V.mark = A.mark;
  int32_t s = 0;
  LG_TRY(lg::launch_adj_check(V, w, order, rows, n_rows, st), "pruned adjacency check");
  LG_TRY(hipMemcpyAsync(&s, w + A.ctrl, sizeof(int32_t), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync(status)");
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s != 0)
    return fail(LINGAM_E_INVALID,
                "order is not a permutation of 0 .. d-1, or a row index is outside [0, n_rows)");
  LG_TRY(lg::launch_adjacency_pruned(A, w, X, ldx, rows, order, max_active, B, st),
         "pruned adjacency launch");
  LG_TRY(hipMemcpyAsync(&s, w + A.ctrl, sizeof(int32_t), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync(status)");
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s != 0)
    return fail(LINGAM_E_DEGENERATE,
                "non-finite data or a correlation matrix that is not positive definite");
  return LINGAM_OK;
}

size_t lingam_total_effects_workspace_size(int64_t d) {
  if (d < 1 || d > kMaxD) return 0;
  return lg::make_effects_layout(d).total;
}

int lingam_total_effects(const double* B, int64_t d, const int32_t* order, double* T, void* ws,
                         size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!B || !order || !T) return fail(LINGAM_E_INVALID, "B, order and T must be non-NULL");
  if (d < 1) return fail(LINGAM_E_INVALID, "need d >= 1 (got %lld)", (long long)d);
  if (d > kMaxD) return fail(LINGAM_E_UNSUPPORTED, "d <= %lld supported", (long long)kMaxD);
  if (T == B) return fail(LINGAM_E_INVALID, "T must not alias B");
  const lg::EffectsLayout A = lg::make_effects_layout(d);
  if (!ws || ws_bytes < A.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", A.total,
                ws ? ws_bytes : (size_t)0);
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  lg::AdjLayout V{};  // the check's view of the status and mark regions
  V.n = 2;
  V.d = d;
  V.ctrl = A.ctrl;
  V.mark = A.mark;
  int32_t s = 0;
  LG_TRY(lg::launch_adj_check(V, w, order, nullptr, 0, st), "total effects check");
  LG_TRY(hipMemcpyAsync(&s, w + A.ctrl, sizeof(int32_t), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync(status)");
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s != 0) return fail(LINGAM_E_INVALID, "order is not a permutation of 0 .. d-1");
  LG_TRY(lg::launch_total_effects(A, w, B, order, T, st), "total effects");
  return LINGAM_OK;
}

int lingam_bootstrap_accumulate(const int32_t* order, const double* B, int64_t d,
                                double threshold, int32_t* order_count, int32_t* edge_count,
                                double* coef_sum, void* stream) {
  g_err[0] = 0;
  if (!order || !B || !order_count || !edge_count)
    return fail(LINGAM_E_INVALID, "order, B, order_count and edge_count must be non-NULL");
  if (d < 1) return fail(LINGAM_E_INVALID, "need d >= 1 (got %lld)", (long long)d);
  if (d > kMaxD) return fail(LINGAM_E_UNSUPPORTED, "d <= %lld supported", (long long)kMaxD);
  if (!(threshold >= 0.0)) return fail(LINGAM_E_INVALID, "threshold must be >= 0");
  LG_TRY(lg::launch_boot_accumulate(order, B, (int)d, threshold, order_count, edge_count,
                                    coef_sum, (hipStream_t)stream),
         "bootstrap accumulate");
  return LINGAM_OK;
}

int lingam_bootstrap_finalize(const int32_t* order_count, const int32_t* edge_count,
                              const double* coef_sum, int64_t d, int32_t n_resamples,
                              double* order_prob, double* edge_prob, double* coef_mean,
                              void* stream) {
  g_err[0] = 0;
  if (!order_count || !edge_count || !order_prob || !edge_prob || (coef_sum && !coef_mean))
    return fail(LINGAM_E_INVALID,
                "order_count, edge_count, order_prob and edge_prob must be non-NULL, and "
                "coef_mean when coef_sum is given");
  if (d < 1) return fail(LINGAM_E_INVALID, "need d >= 1 (got %lld)", (long long)d);
  if (d > kMaxD) return fail(LINGAM_E_UNSUPPORTED, "d <= %lld supported", (long long)kMaxD);
  if (n_resamples < 1)
    return fail(LINGAM_E_INVALID, "need n_resamples >= 1 (got %d)", n_resamples);
  LG_TRY(lg::launch_boot_finalize(order_count, edge_count, coef_sum, (int)d, n_resamples,
                                  order_prob, edge_prob, coef_mean, (hipStream_t)stream),
         "bootstrap finalize");
  return LINGAM_OK;
}

int varlingam_lagged_effects(const double* M, const double* B0, int64_t d, int32_t lags,
                             double* theta, void* stream) {
  g_err[0] = 0;
  if (!M || !B0 || !theta) return fail(LINGAM_E_INVALID, "M, B0 and theta must be non-NULL");
  if (d < 1 || lags < 1)
    return fail(LINGAM_E_INVALID, "need d >= 1 and lags >= 1 (got d=%lld lags=%d)",
                (long long)d, lags);
  if (d > kMaxD || lags > 65535)
    return fail(LINGAM_E_UNSUPPORTED, "d <= %lld and lags <= 65535 supported", (long long)kMaxD);
  if (theta == M) return fail(LINGAM_E_INVALID, "theta must not alias M");
  LG_TRY(lg::launch_lagged_effects(M, B0, (int)d, lags, theta, (hipStream_t)stream),
         "lagged effects");
  return LINGAM_OK;
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
  LG_TRY(lg::launch_residualize_rowmajor(X, n, d, ldx, active, n_active, exo, (char*)ws, st),
         "residualize launch");
  int32_t s = 0;
  LG_TRY(hipMemcpyAsync(&s, ws, sizeof(int32_t), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync(status)");
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (s == LINGAM_E_INVALID) return fail(LINGAM_E_INVALID, "an id in `active` is outside [0, d)");
  if (s != 0) return fail(LINGAM_E_DEGENERATE, "var(x_exo) == 0");
  return LINGAM_OK;
}

size_t lingam_proposer_scores_workspace_size(void) {
  return (sizeof(lg::PropDev) + 255) & ~size_t(255);
}

int lingam_proposer_scores(const float* proposer, const float* features, int64_t rows,
                           float* scores, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!proposer || !features || !scores)
    return fail(LINGAM_E_INVALID, "proposer, features and scores must be non-NULL");
  if (rows < 1 || rows > kMaxN)
    return fail(LINGAM_E_INVALID, "rows %lld outside [1, %lld]", (long long)rows,
                (long long)kMaxN);
  const size_t need = lingam_proposer_scores_workspace_size();
  if (!ws || ws_bytes < need)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", need,
                ws ? ws_bytes : (size_t)0);
  LG_TRY(lg::launch_scores(proposer, features, rows, scores, (char*)ws, (hipStream_t)stream),
         "proposer scores");
  return LINGAM_OK;
}

size_t lingam_proposer_grad_workspace_size(int64_t rows, int32_t n_lists) {
  if (rows < 1 || n_lists < 1 || rows > kMaxN) return 0;
  return lg::make_train_layout(rows, n_lists).total;
}

namespace {

int proposer_grad(const float* proposer, const float* features, int64_t rows,
                  const int64_t* offsets, const int64_t* targets, const float* weights,
                  int32_t n_lists, float* grad, float* loss, float* scores, void* ws,
                  size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!proposer || !features || !offsets || !(targets || weights) || !grad)
    return fail(LINGAM_E_INVALID,
                "proposer, features, offsets, targets (or weights) and grad must be non-NULL");
  if (rows < 1 || rows > kMaxN || n_lists < 1)
    return fail(LINGAM_E_INVALID, "need 1 <= rows <= %lld and n_lists >= 1", (long long)kMaxN);
  const lg::TrainLayout T = lg::make_train_layout(rows, n_lists);
  if (!ws || ws_bytes < T.total)
    return fail(LINGAM_E_WORKSPACE, "workspace of %zu bytes needed (got %zu)", T.total,
                ws ? ws_bytes : (size_t)0);
  hipStream_t st = (hipStream_t)stream;
  LG_TRY(lg::launch_grad(T, proposer, features, offsets, weights ? nullptr : targets, weights,
                         grad, loss, scores, (char*)ws, st),
         "proposer grad");
  int32_t status = 0;
  LG_TRY(hipMemcpyAsync(&status, (char*)ws + T.status, sizeof(int32_t), hipMemcpyDeviceToHost,
                        st),
         "hipMemcpyAsync(status)");
  LG_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (status == 1)
    return fail(LINGAM_E_INVALID,
                weights ? "a list lies outside [0, rows) or has invalid or all-zero weights"
                        : "a list lies outside [0, rows) or a target outside its list");
  if (status == 2)
    return fail(LINGAM_E_INVALID, "non-finite proposer value or feature scale <= 0");
  return LINGAM_OK;
}

}  // namespace

int lingam_proposer_grad(const float* proposer, const float* features, int64_t rows,
                         const int64_t* offsets, const int64_t* targets, int32_t n_lists,
                         float* grad, float* loss, float* scores, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!targets) {
    g_err[0] = 0;
    return fail(LINGAM_E_INVALID, "targets must be non-NULL");
  }
  return proposer_grad(proposer, features, rows, offsets, targets, nullptr, n_lists, grad, loss,
                       scores, ws, ws_bytes, stream);
}

int lingam_proposer_grad_soft(const float* proposer, const float* features, int64_t rows,
                              const int64_t* offsets, const float* weights, int32_t n_lists,
                              float* grad, float* loss, float* scores, void* ws,
                              size_t ws_bytes, void* stream) {
  if (!weights) {
    g_err[0] = 0;
    return fail(LINGAM_E_INVALID, "weights must be non-NULL");
  }
  return proposer_grad(proposer, features, rows, offsets, nullptr, weights, n_lists, grad, loss,
                       scores, ws, ws_bytes, stream);
}

int lingam_proposer_adam(float* proposer, const float* grad, float* m1, float* m2, int32_t step,
                         float lr, float beta1, float beta2, float eps, void* stream) {
  g_err[0] = 0;
  if (!proposer || !grad || !m1 || !m2)
    return fail(LINGAM_E_INVALID, "proposer, grad, m1 and m2 must be non-NULL");
  if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(LINGAM_E_INVALID, "need step >= 1, lr > 0, 0 <= beta < 1, eps > 0");
  const double c1 = 1.0 / (1.0 - pow((double)beta1, (double)step));
  const double c2 = 1.0 / (1.0 - pow((double)beta2, (double)step));
  LG_TRY(lg::launch_adam(proposer, grad, m1, m2, lr, beta1, beta2, eps, (float)c1, (float)c2,
                         (hipStream_t)stream),
         "proposer adam");
  return LINGAM_OK;
}

}  // extern "C"
