// Autotuner of the product launches.
//
// A product is keyed by its arithmetic, shape, batch and operand layout.
// In tuning mode, the first time a key is met on a stream that is not being
// captured, with beta = 0 and an output that overlaps neither operand (so
// that running it again gives the same result), every candidate launch is
// timed with HIP events on that stream and the fastest is stored; the
// product is then run once more with the stored choice, so its result is the
// one every later call gives.  Candidates: the MFMA kernels with the split-K
// count of the heuristic, half, a quarter, double and no split, and the
// general kernel.  Later calls (also inside a graph capture) use the stored
// choice; keys never tuned use the heuristic.  The table lives for the
// process and is shared by every handle.
#include "gemm_internal.h"
#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

namespace ttn {
namespace {

using Key = std::tuple<int, int, int, int, int, int, int, int, int, int, long long, long long, int>;

std::mutex g_mu;
std::map<Key, GemmChoice> g_table;
int g_mode = 0;  // 0: heuristic only, 1: tune new keys, 2: stored choices only

Key key_of(Prec p, const GemmDesc& g) {
  return Key{(int)p, g.M, g.N, g.K, g.K2, g.batch, g.batch1, (int)(g.sAk == 1), (int)(g.sBk == 1),
             (int)(g.beta != 0.0), g.sAm, g.sBn, gemm_members(g)};
}

bool overlaps(const GemmDesc& g) { return g.C == g.A || g.C == g.B; }

float time_once(Prec p, const GemmDesc& g, void* scratch, size_t bytes, hipStream_t s, const GemmChoice& c,
                hipEvent_t e0, hipEvent_t e1, hipError_t* err) {
  *err = hipEventRecord(e0, s);
  if (*err) return 1e30f;
  if (c.path == 0) *err = gemm_mfma(p, g, scratch, bytes, s, c.splits);
  else *err = gemm_plain(p, g, scratch, bytes, s);
  if (*err) return 1e30f;
  if ((*err = hipEventRecord(e1, s))) return 1e30f;
  if ((*err = hipEventSynchronize(e1))) return 1e30f;
  float ms = 0.f;
  *err = hipEventElapsedTime(&ms, e0, e1);
  return ms;
}

// the timing runs are not the product's own launches: kept out of a kernel timer
struct TimerOff {
  KernelTimer* saved;
  TimerOff() : saved(kernel_timer()) { kernel_timer() = nullptr; }
  ~TimerOff() { kernel_timer() = saved; }
};

bool tune(Prec p, const GemmDesc& g, void* scratch, size_t bytes, hipStream_t s, GemmChoice* out) {
  TimerOff off;
  std::vector<GemmChoice> cand;
  int dflt = 0;
  if (gemm_path_mfma_enabled()) {
    // one run with the heuristic gives its split count (and warms the caches)
    hipError_t e = gemm_mfma(p, g, scratch, bytes, s, 0, &dflt);
    if (e == hipSuccess) {
      std::set<int> sp{dflt, std::max(1, dflt / 2), std::max(1, dflt / 4), std::min(128, 2 * dflt), 1};
      for (int x : sp) cand.push_back(GemmChoice{0, x});
    } else if (e != hipErrorNotSupported) {
      return false;
    }
  }
  cand.push_back(GemmChoice{1, 0});
  if (cand.size() == 1) {
    *out = cand[0];
    return true;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return false;
  }
  float best = 1e30f;
  GemmChoice pick = cand[0];
  bool ok = true;
  for (const GemmChoice& c : cand) {
    hipError_t err = hipSuccess;
    float t = 1e30f;
    for (int r = 0; r < 3 && ok; ++r) {
      t = std::min(t, time_once(p, g, scratch, bytes, s, c, e0, e1, &err));
      if (err) ok = false;
    }
    if (!ok) break;
    if (t < best) { best = t; pick = c; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!ok) return false;
  *out = pick;
  return true;
}

}  // namespace

void gemm_tune_set_mode(int mode) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_mode = mode;
}

size_t gemm_tune_entries() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_table.size();
}

void gemm_tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

bool gemm_tuned_choice(Prec prec, const GemmDesc& g, hipStream_t s, void* scratch, size_t scratch_bytes,
                       GemmChoice* out) {
  const Key k = key_of(prec, g);
  int mode;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    mode = g_mode;
    if (mode == 0) return false;
    auto it = g_table.find(k);
    if (it != g_table.end()) {
      *out = it->second;
      return true;
    }
  }
  if (mode != 1 || g.beta != 0.0 || overlaps(g) || g.skip) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  GemmChoice c{0, 0};
  if (!tune(prec, g, scratch, scratch_bytes, s, &c)) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[k] = c;
  *out = c;
  return true;
}

}  // namespace ttn
