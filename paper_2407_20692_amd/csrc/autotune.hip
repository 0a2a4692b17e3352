// Refocus autotuner.  The paper sizes its refocusing blocks from the device
// memory available (Section 4.1); here the batched kernel and its work
// decomposition (planes per work-group, output rows or columns per
// work-group, view-row splits, staged windows) are chosen by timing the
// candidates on the caller's inputs.  Results are kept
// per (shape, device) in memory and, when CPI_AUTOTUNE_CACHE names a file, in
// a text cache of lines "key kp rw splits kernel stages microseconds".
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <algorithm>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "autotune.h"
#include "plan.h"

namespace cpi {

namespace {

std::mutex g_mu;
std::map<std::string, RefocusConfig> g_cache;
bool g_loaded = false;

int log_level() {
  const char* v = std::getenv("CPI_LOG_LEVEL");
  return v ? std::atoi(v) : 0;
}

std::string device_tag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "dev?";
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "dev?";
  std::ostringstream os;
  os << p.gcnArchName << "/cu" << p.multiProcessorCount;
  std::string s = os.str();
  for (char& c : s)
    if (c == ' ' || c == ':') c = '_';
  return s;
}

std::string shape_key(const cpi_geometry* g, int32_t n_alpha) {
  std::ostringstream os;
  os << "wa" << g->wa << "_ha" << g->ha << "_wb" << g->wb << "_hb" << g->hb << "_ow" << g->out_w
     << "_oh" << g->out_h << "_na" << n_alpha << "@" << device_tag();
  return os.str();
}

// Loads the cache file once; a malformed file is ignored as a whole.
void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("CPI_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  if (!f) return;
  std::map<std::string, RefocusConfig> tmp;
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    std::string key;
    RefocusConfig c;
    double us = 0;
    if (!(is >> key >> c.kp >> c.rw >> c.splits >> c.mode >> c.stages >> us) ||
        !refocus_config_supported(c)) {
      if (log_level() > 0)
        std::fprintf(stderr, "cpi: ignoring malformed autotune cache %s\n", path);
      return;
    }
    tmp[key] = c;
  }
  g_cache.insert(tmp.begin(), tmp.end());
}

void store_cache_locked(const std::string& key, const RefocusConfig& c, double us) {
  g_cache[key] = c;
  const char* path = std::getenv("CPI_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  if (f)
    f << key << ' ' << c.kp << ' ' << c.rw << ' ' << c.splits << ' ' << c.mode << ' '
      << c.stages << ' ' << us << '\n';
}

int64_t workgroups(const cpi_geometry* g, int32_t n_alpha, const RefocusConfig& c) {
  const int64_t tx = (g->out_w + 63) / 64;
  const int64_t ty = (g->out_h + c.rw - 1) / c.rw;
  const int64_t gr = (n_alpha + c.kp - 1) / c.kp;
  return tx * ty * gr * c.splits;
}

}  // namespace

// The column-sum kernel with 4 planes x 16 rows and two staged windows, view
// splits until the grid has 8192 work-groups.
RefocusConfig default_sep_config(const cpi_geometry* g, int32_t n_alpha) {
  RefocusConfig c;
  c.mode = 1;
  c.stages = 2;
  c.kp = 4;
  c.rw = g->out_h >= 16 ? 16 : 8;
  c.splits = 1;
  const int max_splits = g->hb < kMaxViewSplits ? g->hb : kMaxViewSplits;
  while (c.splits * 2 <= max_splits && workgroups(g, n_alpha, c) < 8192) c.splits *= 2;
  return c;
}

// Untuned shapes: the row-lane kernel with 8 planes x 32 output columns per
// work-group (the fastest measured on Da 256 x 256, Db 128 x 128); the
// enqueue takes another row-lane shape where the plane set's windows are too
// wide for that one, and the column-sum kernel where none fits.  Views
// narrower than 64 columns take the column-sum kernel.
RefocusConfig default_refocus_config(const cpi_geometry* g, int32_t n_alpha) {
  if (g->wa < 64) return default_sep_config(g, n_alpha);
  RefocusConfig c;
  c.mode = 2;
  c.kp = 8;
  c.rw = 32;
  c.splits = 1;
  c.stages = 2;
  return c;
}

RefocusConfig refocus_config_for(const cpi_geometry* g, int32_t n_alpha) {
  const std::string key = shape_key(g, n_alpha);
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    RefocusConfig c = it->second;
    const int max_splits = g->hb < kMaxViewSplits ? g->hb : kMaxViewSplits;
    if (c.splits > max_splits) c.splits = max_splits;
    return c;
  }
  return default_refocus_config(g, n_alpha);
}

cpi_status autotune_refocus(const float* gamma, const cpi_geometry* g, const double* alphas,
                            int32_t n_alpha, float* out, void* ws, size_t ws_bytes,
                            hipStream_t st, std::string* why) {
  std::vector<RefocusConfig> cands;
  const int max_splits = g->hb < kMaxViewSplits ? g->hb : kMaxViewSplits;
  for (const std::pair<int, int>& t : {std::make_pair(8, 8), std::make_pair(4, 16),
                                       std::make_pair(8, 16), std::make_pair(16, 16),
                                       std::make_pair(8, 32)})
    cands.push_back(RefocusConfig{t.first, t.second, 1, 2, 2});
  for (int mode : {0, 1})
    for (int kp : {1, 2, 4, 8, 16})
      for (int rw : {8, 16, 32})
        for (int sp = 1; sp <= max_splits; sp *= 2) {
          RefocusConfig c{kp, rw, sp, mode, 3};
          if (!refocus_config_supported(c)) continue;
          // one plane x 16 rows and two planes x 32 rows: the staged windows
          // leave a CU four waves (measured 20-50x slower); not searched
          if ((kp == 1 && rw == 16) || (kp == 2 && rw == 32)) continue;
          if (kp > 4 && kp / 2 >= n_alpha) continue;        // planes beyond n_alpha
          if (rw > 8 && rw / 2 >= g->out_h) continue;       // rows beyond out_h
          cands.push_back(c);
        }
  if (g->wa < 2 || g->ha < 2) cands.clear();
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (why) *why = "autotune: cannot create events";
    return CPI_ERR_DEVICE;
  }
  RefocusConfig best = default_refocus_config(g, n_alpha);
  double best_us = 1e300;
  // Times one candidate (a warm-up call, then the mean of 3); < 0 if it
  // cannot run here.
  auto time_of = [&](const RefocusConfig& c, double* us) -> cpi_status {
    *us = -1.0;
    cpi_status s = refocus_enqueue(gamma, g, alphas, n_alpha, out, ws, ws_bytes, st, &c, false);
    if (s != CPI_OK) return CPI_OK;
    const int reps = 3;
    hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r)
      refocus_enqueue(gamma, g, alphas, n_alpha, out, ws, ws_bytes, st, &c, false);
    hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) {
      if (why) *why = "autotune: device failure while timing";
      return CPI_ERR_DEVICE;
    }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    *us = 1000.0 * ms / reps;
    if (log_level() > 1)
      std::fprintf(stderr, "cpi: autotune kernel=%d stages=%d kp=%d rw=%d splits=%d %.1f us\n",
                   c.mode, c.mode ? c.stages : 0, c.kp, c.rw, c.splits, *us);
    return CPI_OK;
  };
  // Phase 1: every shape and split count of both kernels (column sums with
  // three stages); phase 2: the three fastest column-sum candidates with two
  // and four stages.
  std::vector<std::pair<double, RefocusConfig>> sep_times;
  cpi_status fail = CPI_OK;
  for (const RefocusConfig& c : cands) {
    double us;
    fail = time_of(c, &us);
    if (fail != CPI_OK) break;
    if (us < 0) continue;
    if (c.mode == 1) sep_times.push_back({us, c});
    if (us < best_us) {
      best_us = us;
      best = c;
    }
  }
  if (fail == CPI_OK) {
    std::sort(sep_times.begin(), sep_times.end(),
              [](const std::pair<double, RefocusConfig>& a,
                 const std::pair<double, RefocusConfig>& b) { return a.first < b.first; });
    for (size_t k = 0; k < sep_times.size() && k < 3 && fail == CPI_OK; ++k)
      for (int stg : {2, 4}) {
        RefocusConfig c = sep_times[k].second;
        c.stages = stg;
        double us;
        fail = time_of(c, &us);
        if (fail != CPI_OK) break;
        if (us >= 0 && us < best_us) {
          best_us = us;
          best = c;
        }
      }
  }
  if (fail != CPI_OK) {
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return fail;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    store_cache_locked(shape_key(g, n_alpha), best, best_us);
  }
  cpi_status s = refocus_enqueue(gamma, g, alphas, n_alpha, out, ws, ws_bytes, st, &best, false);
  if (s != CPI_OK) return s;
  if (hipStreamSynchronize(st) != hipSuccess) {
    if (why) *why = "autotune: device failure";
    return CPI_ERR_DEVICE;
  }
  return CPI_OK;
}

}  // namespace cpi
