// Stage profiler: optional HIP events around every stage launch, recorded on
// the stream the stage runs on, accumulated per stage on read. With FFC_ROCTX=1
// in the environment every stage is also a roctx range ("ffc:<stage>"), which
// rocprofv3 --marker-trace records beside the kernel trace; the roctx runtime
// is then loaded on first use (the library does not link it otherwise).
#include <dlfcn.h>

#include <cstdlib>
#include <mutex>

#include "ffc_internal.h"

namespace ffc {
namespace {

using PushFn = int (*)(const char*);
using PopFn = int (*)();
struct Roctx {
  PushFn push = nullptr;
  PopFn pop = nullptr;
};

const Roctx& roctx() {
  static const Roctx r = [] {
    Roctx out;
    const char* e = std::getenv("FFC_ROCTX");
    if (!e || e[0] != '1') return out;
    void* h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_GLOBAL);
    if (!h) return out;
    out.push = reinterpret_cast<PushFn>(dlsym(h, "roctxRangePushA"));
    out.pop = reinterpret_cast<PopFn>(dlsym(h, "roctxRangePop"));
    if (!out.push || !out.pop) out = Roctx{};
    return out;
  }();
  return r;
}

struct Pending {
  int stage;
  hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_free;   // recycled events

hipEvent_t get_event() {
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_free.empty()) {
      hipEvent_t e = g_free.back();
      g_free.pop_back();
      return e;
    }
  }
  hipEvent_t e{};
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
std::vector<Pending> g_pending;
double g_ms[FFC_NUM_STAGES] = {};
int64_t g_launches[FFC_NUM_STAGES] = {};

}  // namespace

bool profiling() { return g_on; }

void profiler_release() {
  std::lock_guard<std::mutex> lock(g_mu);
  g_on = false;
  for (const Pending& p : g_pending) {
    (void)hipEventSynchronize(p.stop);
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  g_pending.clear();
  for (hipEvent_t e : g_free) (void)hipEventDestroy(e);
  g_free.clear();
}

const char* const kStageRanges[FFC_NUM_STAGES] = {
    "ffc:tree",  "ffc:sample", "ffc:columns",  "ffc:kblock",  "ffc:cpqr",   "ffc:skel",   "ffc:upward",
    "ffc:evaluate", "ffc:direct", "ffc:solve", "ffc:proposal", "ffc:heldout", "ffc:labels", "ffc:train"};

StageTimer::StageTimer(int stage, hipStream_t st) : stage_(stage), st_(st) {
  if (roctx().push) roctx().push(kStageRanges[stage]);
  if (!g_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;   // not inside graphs
  start_ = get_event();
  stop_ = get_event();
  if (!start_ || !stop_) return;
  active_ = hipEventRecord(start_, st_) == hipSuccess;
}

StageTimer::~StageTimer() {
  if (roctx().pop) roctx().pop();
  if (!active_) return;
  (void)hipEventRecord(stop_, st_);
  std::lock_guard<std::mutex> lock(g_mu);
  g_pending.push_back(Pending{stage_, start_, stop_});
}

}  // namespace ffc

using namespace ffc;

extern "C" {

ffc_status ffc_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_on = on != 0;
  return FFC_OK;
}

ffc_status ffc_profile_read(double* ms_host, int64_t* launches_host, int32_t num_stages, int32_t reset) {
  if (num_stages < 0) {
    set_error("num_stages must be >= 0");
    return FFC_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  for (const Pending& p : g_pending) {
    FFC_HIP_TRY(hipEventSynchronize(p.stop));
    float ms = 0.f;
    FFC_HIP_TRY(hipEventElapsedTime(&ms, p.start, p.stop));
    g_ms[p.stage] += ms;
    g_launches[p.stage] += 1;
    g_free.push_back(p.start);
    g_free.push_back(p.stop);
  }
  g_pending.clear();
  for (int i = 0; i < num_stages && i < FFC_NUM_STAGES; ++i) {
    if (ms_host) ms_host[i] = g_ms[i];
    if (launches_host) launches_host[i] = g_launches[i];
  }
  if (reset) {
    for (int i = 0; i < FFC_NUM_STAGES; ++i) {
      g_ms[i] = 0.0;
      g_launches[i] = 0;
    }
  }
  return FFC_OK;
}

}  // extern "C"

extern "C" ffc_status ffc_autotune_report(int32_t* out_host, int32_t cap, int32_t* count) {
  if (!count || (cap > 0 && !out_host)) {
    ffc::set_error("NULL argument");
    return FFC_ERR_INVALID_ARG;
  }
  *count = ffc::autotune_entries(out_host, cap > 0 ? cap : 0);
  return FFC_OK;
}

extern "C" void ffc_autotune_reset(void) { ffc::autotune_reset(); }
