// Autotuner of the product launches.
//
// A product is keyed by its arithmetic, shape, batch, operand layout and
// launch-group size.  In tuning mode, the first time a key is met on a stream
// that is not being captured, with beta = 0 and an output that overlaps
// neither operand (so that running it again gives the same result), every
// candidate launch shape is timed with HIP events on that stream, three times
// each, and the fastest is stored; the product is then run once more with
// the stored choice.  Candidates: the output tile (float64: 64 x 64, 128 x 64
// or 64 x 128) and the order in which tiles are handed to the XCDs (smaller
// tile dimension fastest, x fastest, y fastest).  No candidate changes the
// arithmetic: the split-K partition is fixed by the shape, and every tile
// issues the same MFMA sequence for an output element, so a tuned launch
// returns the same bits as the default one.  Later calls (also inside a graph
// capture) use the stored choice; keys never tuned use the default.  The
// table lives for the process, is shared by every handle, and can be written
// to and read from a text file (one key and its choice per line).
#include "gemm_internal.h"
#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace ttn {
namespace {

using Key = std::tuple<int, int, int, int, int, int, int, int, int, int, long long, long long, int>;

std::mutex g_mu;
std::map<Key, GemmLaunch> g_table;
int g_mode = 0;  // 0: defaults only, 1: tune new keys, 2: stored choices only

Key key_of(Prec p, const GemmDesc& g) {
  return Key{(int)p, g.M, g.N, g.K, g.K2, g.batch, g.batch1, (int)(g.sAk == 1), (int)(g.sBk == 1),
             (int)(g.beta != 0.0), g.sAm, g.sBn, gemm_members(g)};
}

bool overlaps(const GemmDesc& g) { return g.C == g.A || g.C == g.B; }

float time_once(Prec p, const GemmDesc& g, void* scratch, size_t bytes, hipStream_t s, const GemmLaunch& c,
                hipEvent_t e0, hipEvent_t e1, hipError_t* err) {
  *err = hipEventRecord(e0, s);
  if (*err) return 1e30f;
  *err = gemm_mfma(p, g, scratch, bytes, s, c);
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

bool tune(Prec p, const GemmDesc& g, void* scratch, size_t bytes, hipStream_t s, GemmLaunch* out) {
  TimerOff off;
  // one run with the default launch (warms the caches; products the MFMA
  // kernels do not take have nothing to tune)
  hipError_t e = gemm_mfma(p, g, scratch, bytes, s, GemmLaunch());
  if (e == hipErrorNotSupported) {
    *out = GemmLaunch();
    return true;
  }
  if (e != hipSuccess) return false;
  std::vector<GemmLaunch> cand;
  for (int t = 0; t < (p == P_F64 ? 3 : 1); ++t)
    for (int o = 0; o < 3; ++o) {
      GemmLaunch c;
      c.tile = p == P_F64 ? t + 1 : 0;
      c.orient = o;
      cand.push_back(c);
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return false;
  }
  float best = 1e30f;
  GemmLaunch pick = cand[0];
  bool ok = true;
  for (const GemmLaunch& c : cand) {
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

bool gemm_tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return false;
  for (const auto& kv : g_table) {
    const Key& k = kv.first;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %lld %lld %d : %d %d\n", std::get<0>(k), std::get<1>(k),
                 std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k),
                 std::get<8>(k), std::get<9>(k), std::get<10>(k), std::get<11>(k), std::get<12>(k), kv.second.tile,
                 kv.second.orient);
  }
  return std::fclose(f) == 0;
}

int gemm_tune_load(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  std::map<Key, GemmLaunch> add;
  int v[13];
  long long sa = 0, sb = 0;
  GemmLaunch c;
  int got;
  while ((got = std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %lld %lld %d : %d %d", &v[0], &v[1], &v[2], &v[3],
                            &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &sa, &sb, &v[12], &c.tile, &c.orient)) == 15) {
    if (c.tile < 0 || c.tile > 3) break;
    if (c.orient < 0 || c.orient > 2) break;
    add[Key{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9], sa, sb, v[12]}] = c;
  }
  const bool clean = got == EOF;
  std::fclose(f);
  if (!clean) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : add) g_table[kv.first] = kv.second;
  return (int)add.size();
}

bool gemm_tuned_choice(Prec prec, const GemmDesc& g, hipStream_t s, void* scratch, size_t scratch_bytes,
                       GemmLaunch* out) {
  // symmetric outputs launch their one shape (64 x 64 tiles of the upper
  // triangle) and are not tuned
  if (g.tri) return false;
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
  GemmLaunch c;
  if (!tune(prec, g, scratch, scratch_bytes, s, &c)) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[k] = c;
  *out = c;
  return true;
}

}  // namespace ttn
