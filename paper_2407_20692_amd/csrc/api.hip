// C ABI of the CPI library (declared in include/cpi.h).
//
// Every entry point validates its arguments on the host, then only enqueues
// kernels on the caller's stream.  No entry point allocates device memory:
// all scratch lives in the caller's workspace, laid out by plan.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "autotune.h"
#include "cpi.h"
#include "errors.h"
#include "kernels.h"
#include "plan.h"

namespace {

thread_local std::string g_last_error;

// ---- kernel timing ---------------------------------------------------------
struct ProfRec {
  std::string group;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

void prof_clear_locked() {
  for (ProfRec& r : g_prof) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  g_prof.clear();
}

// Brackets the kernels enqueued during its lifetime with two events.
class ProfScope {
 public:
  ProfScope(const char* group, hipStream_t s) : s_(s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    ProfRec r;
    r.group = group;
    if (hipEventCreate(&r.a) != hipSuccess) return;
    if (hipEventCreate(&r.b) != hipSuccess) {
      hipEventDestroy(r.a);
      return;
    }
    if (hipEventRecord(r.a, s_) != hipSuccess) {
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
      return;
    }
    idx_ = int64_t(g_prof.size());
    g_prof.push_back(r);
  }
  ~ProfScope() {
    if (idx_ < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (idx_ < int64_t(g_prof.size())) hipEventRecord(g_prof[size_t(idx_)].b, s_);
  }
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  hipStream_t s_;
  int64_t idx_ = -1;
};

cpi_status set_error(cpi_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

cpi_status device_error(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_error(CPI_ERR_DEVICE, m);
}

}  // namespace

namespace cpi {
cpi_status report_error(cpi_status s, const std::string& msg) { return set_error(s, msg); }
}  // namespace cpi

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

template <typename F>
cpi_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::exception& e) {
    return set_error(CPI_ERR_DEVICE, std::string("internal error: ") + e.what());
  } catch (...) {
    return set_error(CPI_ERR_DEVICE, "internal error");
  }
}

#define CPI_HIP(call, what)                      \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return device_error(e_, what); \
  } while (0)

cpi::RefGeom ref_geom(const cpi_geometry* g) {
  cpi::RefGeom r;
  r.wa = g->wa;
  r.ha = g->ha;
  r.wb = g->wb;
  r.hb = g->hb;
  r.out_w = g->out_w;
  r.out_h = g->out_h;
  r.mag_x = g->mag_x;
  r.mag_y = g->mag_y;
  r.ca_x = g->ca_x;
  r.ca_y = g->ca_y;
  r.cb_x = g->cb_x;
  r.cb_y = g->cb_y;
  return r;
}

// Enqueue the whole exact correlation for one set of frames.
//   sums_ws: int64 sums in the workspace (raw values, pa_pad / pb_pad long)
cpi_status enqueue_correlate(const cpi::CorrPlan& pl, const uint8_t* fa, const uint8_t* fb,
                             uint8_t* ws, int layout, double* gamma, float* gamma_f32,
                             int64_t* numer, hipStream_t st) {
  int64_t* sum_a = reinterpret_cast<int64_t*>(ws + pl.off_sum_a);
  int64_t* sum_b = reinterpret_cast<int64_t*>(ws + pl.off_sum_b);
  uint32_t* stats = reinterpret_cast<uint32_t*>(ws + pl.off_stats);
  uint8_t* op_a = ws + pl.off_op_a;
  uint8_t* op_b = ws + pl.off_op_b;
  int64_t* sum2_a = reinterpret_cast<int64_t*>(ws + pl.off_sum2_a);
  int64_t* sum2_b = reinterpret_cast<int64_t*>(ws + pl.off_sum2_b);
  {
    // popcount sums, the 64 flag words and (byte frames) the byte sums
    cpi::ZeroRanges z;
    z.add(sum_a, pl.pa_pad);
    z.add(sum_b, pl.pb_pad);
    z.add(stats, 32);
    if (pl.fmt != CPI_FRAMES_BIT1) {
      z.add(sum2_a, pl.pa_pad);
      z.add(sum2_b, pl.pb_pad);
    }
    CPI_HIP(cpi::zero_ranges(z, st), "fill");
  }

  cpi::GemmArgs g;
  g.opm = op_b;
  g.opn = op_a;
  g.m_pad = pl.pb_pad;
  g.n_pad = pl.pa_pad;
  g.layout = layout;
  g.pa = pl.pa;
  g.pb = pl.pb;
  g.n = pl.n;
  g.sum_a = sum_a;
  g.sum_b = sum_b;
  g.stats = stats;
  g.gamma = gamma;
  g.gamma_f32 = gamma_f32;
  g.numer = numer;

  // matrix-core encoding of the bit contraction, decided once for this call:
  // FP4 needs the M rows (detector B) with bits 0 and 2 of each group swapped
  const bool fp4 = cpi::bits_use_fp4(pl.kpad_bits / cpi::kBitBlock);
  if (pl.fmt == CPI_FRAMES_BIT1) {
    {
      ProfScope ps("ingest", st);
      const cpi::IngestJob ja{fa, pl.pa, pl.pa_pad, op_a, sum_a, nullptr, 0};
      const cpi::IngestJob jb{fb, pl.pb, pl.pb_pad, op_b, sum_b, nullptr, fp4 ? 1 : 0};
      CPI_HIP(cpi::ingest_bits(ja, jb, pl.n, pl.kpad_bits, st), "ingest");
    }
    g.row_bytes = pl.row_bytes_bits;
    g.kblocks = pl.kpad_bits / cpi::kBitBlock;
    g.fp4 = fp4 ? 1 : 0;
    g.mode = cpi::EPI_FINAL;
    ProfScope ps("gemm", st);
    CPI_HIP(cpi::gemm_correlate(g, true, st), "gemm");
    return CPI_OK;
  }

  // Byte frames: one pass builds bit rows, popcounts and the OR of all bytes.
  // Binary data (OR <= 1) is then complete; otherwise the device also runs
  // the byte-sum and int8-row passes and the byte contraction, and skips the
  // bit contraction.  Both branches are enqueued; no host synchronisation.
  {
    ProfScope ps("ingest", st);
    const cpi::IngestJob ja{fa, pl.pa, pl.pa_pad, op_a, sum_a, sum2_a, 0};
    const cpi::IngestJob jb{fb, pl.pb, pl.pb_pad, op_b, sum_b, sum2_b, fp4 ? 1 : 0};
    CPI_HIP(cpi::u8_to_bits(ja, jb, pl.n, pl.kpad_bits, stats, st), "ingest");
    CPI_HIP(cpi::u8_sums(ja, jb, pl.n, stats, st), "sums");
    CPI_HIP(cpi::u8_to_bytes(ja, jb, pl.n, pl.kpad_bytes, stats, st), "ingest");
  }

  ProfScope ps("gemm", st);
  cpi::GemmArgs gb = g;
  gb.row_bytes = pl.row_bytes_bits;
  gb.kblocks = pl.kpad_bits / cpi::kBitBlock;
  gb.mode = cpi::EPI_FINAL;
  gb.cond = 1;
  gb.fp4 = fp4 ? 1 : 0;
  CPI_HIP(cpi::gemm_correlate(gb, true, st), "gemm");

  cpi::GemmArgs gy = g;
  gy.row_bytes = pl.row_bytes_bytes;
  gy.cond = 2;
  gy.offset_from_stats = 1;
  gy.sum_a = sum2_a;
  gy.sum_b = sum2_b;
  gy.acc64 = reinterpret_cast<int64_t*>(ws + pl.off_acc64);
  for (int pass = 0; pass < pl.passes; ++pass) {
    const int64_t k0 = int64_t(pass) * cpi::kByteChunk;
    int64_t k1 = k0 + cpi::kByteChunk;
    if (k1 > pl.kpad_bytes) k1 = pl.kpad_bytes;
    gy.k_byte_off = k0;
    gy.kblocks = (k1 - k0) / cpi::kByteBlock;
    if (pl.passes == 1)
      gy.mode = cpi::EPI_FINAL;
    else if (pass == 0)
      gy.mode = cpi::EPI_STORE64;
    else if (pass + 1 < pl.passes)
      gy.mode = cpi::EPI_ADD64;
    else
      gy.mode = cpi::EPI_FINAL_ACC64;
    CPI_HIP(cpi::gemm_correlate(gy, false, st), "gemm");
  }
  return CPI_OK;
}

cpi_status check_frames(const void* a, const void* b) {
  if (!a || !b) return set_error(CPI_ERR_INVALID_ARG, "frame pointers must not be null");
  if (!aligned16(a) || !aligned16(b))
    return set_error(CPI_ERR_INVALID_ARG, "frame pointers must be 16-byte aligned");
  return CPI_OK;
}

cpi_status check_refocus_args(const float* gamma, const cpi_geometry* g, const double* alphas,
                              int32_t n_alpha, float* out, void* ws, size_t ws_bytes,
                              cpi::RefocusPlan* pl) {
  std::string why;
  cpi_status s = cpi::plan_refocus(g, n_alpha, pl, &why);
  if (s != CPI_OK) return set_error(s, why);
  s = cpi::validate_alphas(g, alphas, n_alpha, &why);
  if (s != CPI_OK) return set_error(s, why);
  if (!gamma || !out || !ws) return set_error(CPI_ERR_INVALID_ARG, "null device pointer");
  if (!aligned16(gamma) || !aligned16(out) || !aligned16(ws))
    return set_error(CPI_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
  if (ws_bytes < pl->total)
    return set_error(CPI_ERR_WORKSPACE, "refocus workspace too small: need " +
                                            std::to_string(pl->total) + " bytes");
  return CPI_OK;
}

cpi_status enqueue_tables(const cpi_geometry* g, const double* alphas, int32_t n_alpha,
                          const cpi::RefocusPlan& pl, uint8_t* ws, hipStream_t st) {
  const cpi::RefGeom rg = ref_geom(g);
  int32_t* itab = reinterpret_cast<int32_t*>(ws + pl.off_itab);
  float* ftab = reinterpret_cast<float*>(ws + pl.off_ftab);
  ProfScope ps("refocus_tables", st);
  for (int first = 0; first < n_alpha; first += cpi::kAlphaPerLaunch) {
    const int cnt = (n_alpha - first) < cpi::kAlphaPerLaunch ? n_alpha - first : cpi::kAlphaPerLaunch;
    CPI_HIP(cpi::refocus_tables(rg, alphas, first, cnt, pl.table_stride, itab, ftab,
                                ws + pl.off_ytab, st),
            "refocus tables");
  }
  return CPI_OK;
}

}  // namespace

namespace cpi {

// Shared by the public refocus entry points and the autotuner.
cpi_status refocus_enqueue(const float* gamma, const cpi_geometry* g, const double* alphas,
                           int32_t n_alpha, float* out, void* workspace, size_t ws_bytes,
                           hipStream_t st, const RefocusConfig* forced, bool plain) {
  RefocusPlan pl;
  cpi_status s = check_refocus_args(gamma, g, alphas, n_alpha, out, workspace, ws_bytes, &pl);
  if (s != CPI_OK) return s;
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  s = enqueue_tables(g, alphas, n_alpha, pl, ws, st);
  if (s != CPI_OK) return s;
  const RefGeom rg = ref_geom(g);
  const int32_t* itab = reinterpret_cast<const int32_t*>(ws + pl.off_itab);
  const float* ftab = reinterpret_cast<const float*>(ws + pl.off_ftab);
  if (plain || g->wa < 2 || g->ha < 2) {
    ProfScope ps("refocus_plain", st);
    for (int k = 0; k < n_alpha; ++k)
      CPI_HIP(refocus_plain(gamma, rg, itab, ftab, pl.table_stride, k, out, st), "refocus");
    return CPI_OK;
  }
  RefocusConfig c = forced ? *forced : refocus_config_for(g, n_alpha);
  float* partial = reinterpret_cast<float*>(ws + pl.off_partial);
  if (c.mode == 2 && !forced && !rows_supported(rg, alphas, n_alpha, c.kp, c.rw, pl.rows_chunk)) {
    // the configured row-lane shape does not take this plane set: the next
    // shape whose windows hold it, in order of pairs per work-group
    for (const auto& t : {std::make_pair(8, 32), std::make_pair(16, 16), std::make_pair(8, 16),
                          std::make_pair(16, 8), std::make_pair(8, 8), std::make_pair(4, 16)})
      if (rows_supported(rg, alphas, n_alpha, t.first, t.second, pl.rows_chunk)) {
        c.kp = t.first;
        c.rw = t.second;
        break;
      }
  }
  if (c.mode == 2) {
    if (rows_supported(rg, alphas, n_alpha, c.kp, c.rw, pl.rows_chunk)) {
      RowsWorkspace w;
      w.xe = reinterpret_cast<int32_t*>(ws + pl.off_rows_xe);
      w.yr = reinterpret_cast<int2*>(ws + pl.off_rows_yr);
      w.t = partial;
      w.chunk = int(pl.rows_chunk);
      w.wout_cap = pl.rows_wout_cap;
      ProfScope ps("refocus_batched", st);
      CPI_HIP(refocus_rows(gamma, rg, alphas, itab, ftab, ws + pl.off_ytab, pl.table_stride,
                           n_alpha, c.kp, c.rw, w, out, st),
              "refocus");
      return CPI_OK;
    }
    if (forced)
      return set_error(CPI_ERR_UNSUPPORTED,
                       "row-lane refocus does not take this geometry or plane set");
    c = default_sep_config(g, n_alpha);
  }
  ProfScope ps("refocus_batched", st);
  CPI_HIP(refocus_batched(gamma, rg, itab, ftab, ws + pl.off_ytab, ws + pl.off_bounds,
                          pl.table_stride, n_alpha, c, partial, out, st),
          "refocus");
  return CPI_OK;
}

// Enqueue with an explicit batched configuration against a workspace of
// `ws_bytes`, which must hold the tables and that configuration's partial
// sums (not the whole cpi_refocus_workspace_size).  Column-sum and per-row
// kernels only.
cpi_status refocus_enqueue_config(const float* gamma, const cpi_geometry* g, const double* alphas,
                                  int32_t n_alpha, float* out, void* workspace, size_t ws_bytes,
                                  hipStream_t st, const RefocusConfig& c) {
  RefocusPlan pl;
  std::string why;
  cpi_status s = plan_refocus(g, n_alpha, &pl, &why);
  if (s != CPI_OK) return set_error(s, why);
  s = validate_alphas(g, alphas, n_alpha, &why);
  if (s != CPI_OK) return set_error(s, why);
  if (!gamma || !out || !workspace) return set_error(CPI_ERR_INVALID_ARG, "null device pointer");
  if (!aligned16(gamma) || !aligned16(out) || !aligned16(workspace))
    return set_error(CPI_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
  if (c.mode == 2 || !refocus_config_supported(c))
    return set_error(CPI_ERR_UNSUPPORTED, "refocus configuration is not built");
  const int sp = std::min<int>(c.splits, g->hb);
  const size_t need =
      pl.off_partial +
      (sp > 1 ? size_t(sp) * size_t(n_alpha) * size_t(g->out_w) * size_t(g->out_h) * 4 : 0);
  if (ws_bytes < need)
    return set_error(CPI_ERR_WORKSPACE, "refocus workspace too small: need " +
                                            std::to_string(need) + " bytes");
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  s = enqueue_tables(g, alphas, n_alpha, pl, ws, st);
  if (s != CPI_OK) return s;
  const RefGeom rg = ref_geom(g);
  const int32_t* itab = reinterpret_cast<const int32_t*>(ws + pl.off_itab);
  const float* ftab = reinterpret_cast<const float*>(ws + pl.off_ftab);
  if (g->wa < 2 || g->ha < 2) {
    ProfScope ps("refocus_plain", st);
    for (int k = 0; k < n_alpha; ++k)
      CPI_HIP(refocus_plain(gamma, rg, itab, ftab, pl.table_stride, k, out, st), "refocus");
    return CPI_OK;
  }
  ProfScope ps("refocus_batched", st);
  CPI_HIP(refocus_batched(gamma, rg, itab, ftab, ws + pl.off_ytab, ws + pl.off_bounds,
                          pl.table_stride, n_alpha, c,
                          reinterpret_cast<float*>(ws + pl.off_partial), out, st),
          "refocus");
  return CPI_OK;
}

}  // namespace cpi

namespace {

// Workspace of cpi_refocus_noalloc: one array per device, kept for the life
// of the process, found once per device through its symbol address (the
// array's name in host code is not its device address).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

cpi_status noalloc_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(CPI_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(CPI_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(CPI_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return CPI_OK;
}

}  // namespace

extern "C" {

const char* cpi_version(void) { return "cpi-mi355x 0.1.0 (gfx950)"; }

const char* cpi_status_string(cpi_status s) {
  switch (s) {
    case CPI_OK: return "CPI_OK";
    case CPI_ERR_INVALID_ARG: return "CPI_ERR_INVALID_ARG";
    case CPI_ERR_UNSUPPORTED: return "CPI_ERR_UNSUPPORTED";
    case CPI_ERR_OVERFLOW: return "CPI_ERR_OVERFLOW";
    case CPI_ERR_WORKSPACE: return "CPI_ERR_WORKSPACE";
    case CPI_ERR_DEVICE: return "CPI_ERR_DEVICE";
    case CPI_ERR_NOT_READY: return "CPI_ERR_NOT_READY";
  }
  return "CPI_ERR_UNKNOWN";
}

const char* cpi_last_error(void) { return g_last_error.c_str(); }

cpi_status cpi_geometry_default(int32_t wa, int32_t ha, int32_t wb, int32_t hb, cpi_geometry* out) {
  return guarded([&]() -> cpi_status {
    if (!out) return set_error(CPI_ERR_INVALID_ARG, "out is null");
    if (wa <= 0 || ha <= 0 || wb <= 0 || hb <= 0)
      return set_error(CPI_ERR_INVALID_ARG, "sizes must be positive");
    cpi_geometry g;
    g.wa = wa;
    g.ha = ha;
    g.wb = wb;
    g.hb = hb;
    g.mag_x = double(wa) / double(wb);
    g.mag_y = double(ha) / double(hb);
    g.ca_x = (wa - 1) / 2.0;
    g.ca_y = (ha - 1) / 2.0;
    g.cb_x = (wb - 1) / 2.0;
    g.cb_y = (hb - 1) / 2.0;
    g.out_w = wa;
    g.out_h = ha;
    *out = g;
    return CPI_OK;
  });
}

}  // extern "C"

namespace {

// Workspace bytes cpi_correlate may use: the caller's, capped by the
// environment variable CPI_WORKSPACE_LIMIT (a byte count) when it is set.
size_t usable_workspace(size_t given) {
  const char* v = std::getenv("CPI_WORKSPACE_LIMIT");
  if (!v || !*v) return given;
  char* end = nullptr;
  const unsigned long long x = std::strtoull(v, &end, 10);
  if (end == v) return given;
  return size_t(x) < given ? size_t(x) : given;
}

constexpr int64_t kBlockUnit = 512;   // frames; keeps every block 16-byte aligned

// Longer inputs than one ingest pass takes are folded in blocks of at most
// that many frames through the running sums.
using cpi::kMaxPassFrames;
static_assert(kMaxPassFrames % kBlockUnit == 0, "blocks of whole 512-frame units");

// Defined with the streaming calls below; gamma_buffers 0 makes a handle
// whose pushes fold the sums only (the blocks of cpi_correlate).
cpi_status stream_create(int64_t pa, int64_t pb, cpi_frame_format fmt, int64_t max_chunk,
                         int gamma_buffers, void* workspace, size_t bytes, void* stream,
                         cpi_stream_t* out);

// Memory-adaptive blocking: the largest multiple of kBlockUnit frames (at most
// n rounded up) whose running-sum state fits in `bytes`, and that state's
// size; 0 when not even kBlockUnit frames fit.
int64_t block_frames(int64_t n, int64_t pa, int64_t pb, cpi_frame_format fmt, size_t bytes,
                     size_t* need) {
  auto size_for = [&](int64_t units, size_t* b) {
    cpi::StreamPlan sp;
    std::string why;
    if (cpi::plan_stream(pa, pb, int(fmt), units * kBlockUnit, &sp, &why, 0) != CPI_OK)
      return false;
    *b = sp.total;
    return true;
  };
  int64_t lo = 0, hi = (n + kBlockUnit - 1) / kBlockUnit;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    size_t b = 0;
    if (size_for(mid, &b) && b <= bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  if (lo == 0) {
    size_t b = 0;
    *need = size_for(1, &b) ? b : 0;
    return 0;
  }
  size_for(lo, need);
  return lo * kBlockUnit;
}

}  // namespace

extern "C" {

cpi_status cpi_correlate_workspace_size(int64_t n, int64_t pa, int64_t pb, cpi_frame_format fmt,
                                        size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return set_error(CPI_ERR_INVALID_ARG, "bytes is null");
    cpi::CorrPlan pl;
    std::string why;
    cpi_status s = cpi::plan_correlate(n, pa, pb, int(fmt), &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    *bytes = pl.total;
    if (n > kMaxPassFrames) {
      // blocks of kMaxPassFrames frames
      size_t need = 0;
      block_frames(kMaxPassFrames, pa, pb, fmt, SIZE_MAX, &need);
      if (need == 0) return set_error(CPI_ERR_INVALID_ARG, "pa * pb too large for blocked work");
      *bytes = need;
    }
    const size_t limit = usable_workspace(*bytes);
    if (limit < *bytes) {
      size_t need = 0;
      block_frames(n, pa, pb, fmt, limit, &need);
      if (need > 0 && need < *bytes) *bytes = need;
    }
    return CPI_OK;
  });
}

cpi_status cpi_correlate(const void* frames_a, const void* frames_b, int64_t n, int64_t pa,
                         int64_t pb, cpi_frame_format fmt, cpi_gamma_layout layout,
                         double* gamma, float* gamma_f32, int64_t* numer, int64_t* sum_a,
                         int64_t* sum_b, void* workspace, size_t workspace_bytes,
                         void* stream) {
  return guarded([&]() -> cpi_status {
    cpi::CorrPlan pl;
    std::string why;
    cpi_status s = cpi::plan_correlate(n, pa, pb, int(fmt), &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    s = check_frames(frames_a, frames_b);
    if (s != CPI_OK) return s;
    if (layout != CPI_GAMMA_VIEW_MAJOR && layout != CPI_GAMMA_PIXEL_MAJOR)
      return set_error(CPI_ERR_INVALID_ARG, "unknown Gamma layout");
    if (!gamma && !gamma_f32 && !numer)
      return set_error(CPI_ERR_INVALID_ARG, "at least one of gamma, gamma_f32, numer is required");
    const void* outs[5] = {gamma, gamma_f32, numer, sum_a, sum_b};
    for (const void* o : outs)
      if (o && !aligned16(o)) return set_error(CPI_ERR_INVALID_ARG, "outputs must be 16-byte aligned");
    if (!workspace || !aligned16(workspace))
      return set_error(CPI_ERR_INVALID_ARG, "workspace must be a 16-byte aligned device pointer");
    const size_t usable = usable_workspace(workspace_bytes);
    if (usable < pl.total || n > kMaxPassFrames) {
      // memory-adaptive blocking (and inputs longer than one ingest pass):
      // fold the frames in blocks through the running sums of the streaming
      // path (exact, same result)
      size_t need = 0;
      int64_t f = block_frames(n, pa, pb, fmt, usable, &need);
      if (f > kMaxPassFrames) f = kMaxPassFrames;
      if (f == 0)
        return set_error(CPI_ERR_WORKSPACE, "correlate workspace too small: need " +
                                                std::to_string(pl.total) +
                                                " bytes, or at least " + std::to_string(need) +
                                                " to work in blocks of 512 frames");
      cpi_stream_t h = nullptr;
      s = stream_create(pa, pb, fmt, f, 0, workspace, usable, stream, &h);
      if (s != CPI_OK) return s;
      const int64_t fa = cpi::frame_bytes(pa, int(fmt)), fb = cpi::frame_bytes(pb, int(fmt));
      const uint8_t* a8 = static_cast<const uint8_t*>(frames_a);
      const uint8_t* b8 = static_cast<const uint8_t*>(frames_b);
      for (int64_t f0 = 0; f0 < n && s == CPI_OK; f0 += f) {
        const int64_t k = n - f0 < f ? n - f0 : f;
        s = cpi_stream_push(h, a8 + f0 * fa, b8 + f0 * fb, k);
      }
      if (s == CPI_OK) s = cpi_stream_gamma(h, layout, gamma, gamma_f32, numer, sum_a, sum_b);
      const std::string err = s == CPI_OK ? std::string() : std::string(cpi_last_error());
      cpi_stream_destroy(h);
      return s == CPI_OK ? CPI_OK : set_error(s, err);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    s = enqueue_correlate(pl, static_cast<const uint8_t*>(frames_a),
                          static_cast<const uint8_t*>(frames_b), ws, int(layout), gamma,
                          gamma_f32, numer, st);
    if (s != CPI_OK) return s;
    // per-pixel sums: popcounts for bit rows, byte sums for non-binary bytes
    const uint32_t* stats = reinterpret_cast<const uint32_t*>(ws + pl.off_stats);
    const int64_t* s1a = reinterpret_cast<const int64_t*>(ws + pl.off_sum_a);
    const int64_t* s1b = reinterpret_cast<const int64_t*>(ws + pl.off_sum_b);
    const int64_t* s2a = reinterpret_cast<const int64_t*>(ws + pl.off_sum2_a);
    const int64_t* s2b = reinterpret_cast<const int64_t*>(ws + pl.off_sum2_b);
    if (fmt == CPI_FRAMES_BIT1) {
      if (sum_a)
        CPI_HIP(hipMemcpyAsync(sum_a, s1a, size_t(pa) * 8, hipMemcpyDeviceToDevice, st), "copy sums");
      if (sum_b)
        CPI_HIP(hipMemcpyAsync(sum_b, s1b, size_t(pb) * 8, hipMemcpyDeviceToDevice, st), "copy sums");
    } else {
      if (sum_a) CPI_HIP(cpi::select_i64(sum_a, s1a, s2a, pa, stats, st), "copy sums");
      if (sum_b) CPI_HIP(cpi::select_i64(sum_b, s1b, s2b, pb, stats, st), "copy sums");
    }
    return CPI_OK;
  });
}

cpi_status cpi_correlate_f32_plain_workspace_size(int64_t n, int64_t pa, int64_t pb,
                                                  cpi_frame_format fmt, size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return set_error(CPI_ERR_INVALID_ARG, "bytes is null");
    cpi::PlainPlan pl;
    std::string why;
    cpi_status s = cpi::plan_correlate_plain(n, pa, pb, int(fmt), &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    *bytes = pl.total;
    return CPI_OK;
  });
}

cpi_status cpi_correlate_f32_plain(const void* frames_a, const void* frames_b, int64_t n,
                                   int64_t pa, int64_t pb, cpi_frame_format fmt,
                                   cpi_gamma_layout layout, float* gamma_f32, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi::PlainPlan pl;
    std::string why;
    cpi_status s = cpi::plan_correlate_plain(n, pa, pb, int(fmt), &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    s = check_frames(frames_a, frames_b);
    if (s != CPI_OK) return s;
    if (layout != CPI_GAMMA_VIEW_MAJOR && layout != CPI_GAMMA_PIXEL_MAJOR)
      return set_error(CPI_ERR_INVALID_ARG, "unknown Gamma layout");
    if (!gamma_f32 || !aligned16(gamma_f32))
      return set_error(CPI_ERR_INVALID_ARG, "gamma_f32 must be a 16-byte aligned device pointer");
    if (!workspace || !aligned16(workspace))
      return set_error(CPI_ERR_INVALID_ARG, "workspace must be a 16-byte aligned device pointer");
    if (workspace_bytes < pl.total)
      return set_error(CPI_ERR_WORKSPACE,
                       "plain workspace too small: need " + std::to_string(pl.total) + " bytes");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    float* fa = reinterpret_cast<float*>(ws + pl.off_fa);
    float* fb = reinterpret_cast<float*>(ws + pl.off_fb);
    float* sa = reinterpret_cast<float*>(ws + pl.off_sa);
    float* sb = reinterpret_cast<float*>(ws + pl.off_sb);
    {
      ProfScope ps("unpack_f32", st);
      CPI_HIP(cpi::fill_u32(reinterpret_cast<uint32_t*>(sa), pl.pa_pad, 0, st), "fill");
      CPI_HIP(cpi::fill_u32(reinterpret_cast<uint32_t*>(sb), pl.pb_pad, 0, st), "fill");
      CPI_HIP(cpi::unpack_f32(static_cast<const uint8_t*>(frames_a), int(fmt), n, pa, pl.kpad,
                              pl.pa_pad, fa, sa, st),
              "unpack");
      CPI_HIP(cpi::unpack_f32(static_cast<const uint8_t*>(frames_b), int(fmt), n, pb, pl.kpad,
                              pl.pb_pad, fb, sb, st),
              "unpack");
    }
    ProfScope ps("sgemm_f32", st);
    CPI_HIP(cpi::sgemm_gamma(fb, fa, pl.kpad, pl.pb_pad, pl.pa_pad, pa, pb, n, sa, sb,
                             int(layout), gamma_f32, st),
            "sgemm");
    return CPI_OK;
  });
}

cpi_status cpi_refocus_workspace_size(const cpi_geometry* g, int32_t n_alpha, size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return set_error(CPI_ERR_INVALID_ARG, "bytes is null");
    cpi::RefocusPlan pl;
    std::string why;
    cpi_status s = cpi::plan_refocus(g, n_alpha, &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    *bytes = pl.total;
    return CPI_OK;
  });
}

cpi_status cpi_refocus(const float* gamma, const cpi_geometry* g, const double* alphas,
                       int32_t n_alpha, float* out, void* workspace, size_t workspace_bytes,
                       void* stream) {
  return guarded([&]() -> cpi_status {
    return cpi::refocus_enqueue(gamma, g, alphas, n_alpha, out, workspace, workspace_bytes,
                                static_cast<hipStream_t>(stream), nullptr, false);
  });
}

cpi_status cpi_refocus_noalloc(const float* gamma, const cpi_geometry* g, const double* alphas,
                               int32_t n_alpha, float* out, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi::RefocusPlan pl;
    std::string why;
    cpi_status s = cpi::plan_refocus(g, n_alpha, &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    // The configuration cpi_refocus would take, restricted to the kernels
    // whose workspace is the tables plus split partial sums, with view-row
    // splits halved until that fits the scratch array.
    cpi::RefocusConfig c = cpi::refocus_config_for(g, n_alpha);
    if (c.mode == 2) c = cpi::default_sep_config(g, n_alpha);
    auto need = [&](const cpi::RefocusConfig& k) {
      const int sp = std::min<int>(k.splits, g->hb);
      return pl.off_partial + (sp > 1 ? size_t(sp) * size_t(n_alpha) * size_t(g->out_w) *
                                            size_t(g->out_h) * 4
                                      : 0);
    };
    while (c.splits > 1 && need(c) > kNoAllocScratchBytes) c.splits /= 2;
    if (need(c) > kNoAllocScratchBytes)
      return set_error(CPI_ERR_WORKSPACE,
                       "refocus needs " + std::to_string(need(c)) +
                           " bytes of workspace; the allocation-free entry point has " +
                           std::to_string(kNoAllocScratchBytes));
    void* ws = nullptr;
    s = noalloc_scratch(&ws);
    if (s != CPI_OK) return s;
    return cpi::refocus_enqueue_config(gamma, g, alphas, n_alpha, out, ws, need(c),
                                       static_cast<hipStream_t>(stream), c);
  });
}

cpi_status cpi_refocus_plain(const float* gamma, const cpi_geometry* g, const double* alphas,
                             int32_t n_alpha, float* out, void* workspace,
                             size_t workspace_bytes, void* stream) {
  return guarded([&]() -> cpi_status {
    return cpi::refocus_enqueue(gamma, g, alphas, n_alpha, out, workspace, workspace_bytes,
                                static_cast<hipStream_t>(stream), nullptr, true);
  });
}

cpi_status cpi_autotune_refocus(const float* gamma, const cpi_geometry* g, const double* alphas,
                                int32_t n_alpha, float* out, void* workspace,
                                size_t workspace_bytes, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi::RefocusPlan pl;
    cpi_status s = check_refocus_args(gamma, g, alphas, n_alpha, out, workspace, workspace_bytes, &pl);
    if (s != CPI_OK) return s;
    std::string why;
    s = cpi::autotune_refocus(gamma, g, alphas, n_alpha, out, workspace, workspace_bytes,
                              static_cast<hipStream_t>(stream), &why);
    if (s != CPI_OK) return set_error(s, why);
    return CPI_OK;
  });
}

cpi_status cpi_refocus_config(const cpi_geometry* g, int32_t n_alpha, int32_t* planes_per_group,
                              int32_t* rows_per_wave, int32_t* view_splits) {
  return guarded([&]() -> cpi_status {
    cpi::RefocusPlan pl;
    std::string why;
    cpi_status s = cpi::plan_refocus(g, n_alpha, &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    if (!planes_per_group || !rows_per_wave || !view_splits)
      return set_error(CPI_ERR_INVALID_ARG, "null argument");
    const cpi::RefocusConfig c = cpi::refocus_config_for(g, n_alpha);
    *planes_per_group = c.kp;
    *rows_per_wave = c.rw;
    *view_splits = c.splits;
    return CPI_OK;
  });
}

cpi_status cpi_refocus_get_tiles(const cpi_geometry* g, int32_t n_alpha, cpi_refocus_tiles* out) {
  return guarded([&]() -> cpi_status {
    cpi::RefocusPlan pl;
    std::string why;
    cpi_status s = cpi::plan_refocus(g, n_alpha, &pl, &why);
    if (s != CPI_OK) return set_error(s, why);
    if (!out) return set_error(CPI_ERR_INVALID_ARG, "null argument");
    const cpi::RefocusConfig c = cpi::refocus_config_for(g, n_alpha);
    out->planes_per_group = c.kp;
    out->rows_per_wave = c.rw;
    out->view_splits = c.splits;
    out->kernel = c.mode;
    out->stages = c.mode == 1 ? c.stages : 0;
    return CPI_OK;
  });
}

cpi_status cpi_refocus_tiled(const float* gamma, const cpi_geometry* g, const double* alphas,
                             int32_t n_alpha, float* out, const cpi_refocus_tiles* tiles,
                             void* workspace, size_t workspace_bytes, void* stream) {
  return guarded([&]() -> cpi_status {
    if (!tiles) return set_error(CPI_ERR_INVALID_ARG, "null tiles");
    cpi::RefocusConfig c;
    c.kp = tiles->planes_per_group;
    c.rw = tiles->rows_per_wave;
    c.splits = tiles->view_splits;
    c.mode = tiles->kernel;
    c.stages = tiles->stages;
    if (!cpi::refocus_config_supported(c))
      return set_error(CPI_ERR_UNSUPPORTED, "refocus configuration is not built");
    return cpi::refocus_enqueue(gamma, g, alphas, n_alpha, out, workspace, workspace_bytes,
                                static_cast<hipStream_t>(stream), &c, false);
  });
}

}  // extern "C"

namespace {

// Geometry under which refocusing the resampled views (view j * nx + i at
// lens-plane point (ox + i sx, oy + j sy)) is refocusing with that sample
// grid: (1 - alpha) M (x_b - c_b) = (1 - alpha) (M sx) (i - (c_b - ox) / sx).
cpi_status lens_geometry(const cpi_geometry* g, const cpi_lens_sampling* s, cpi_geometry* gs) {
  if (!g || !s || !gs) return set_error(CPI_ERR_INVALID_ARG, "null argument");
  if (s->nx < 1 || s->ny < 1 || s->nx > 65536 || s->ny > 65536)
    return set_error(CPI_ERR_INVALID_ARG, "sample counts must be in [1, 65536]");
  const double v[4] = {s->ox, s->oy, s->sx, s->sy};
  for (double x : v)
    if (!std::isfinite(x) || std::fabs(x) > 1048576.0)
      return set_error(CPI_ERR_INVALID_ARG, "sample grid parameters must be finite and below 2^20");
  if (!(s->sx > 0.0) || !(s->sy > 0.0))
    return set_error(CPI_ERR_INVALID_ARG, "sample spacings must be positive");
  *gs = *g;
  gs->wb = s->nx;
  gs->hb = s->ny;
  gs->mag_x = g->mag_x * s->sx;
  gs->mag_y = g->mag_y * s->sy;
  gs->cb_x = (g->cb_x - s->ox) / s->sx;
  gs->cb_y = (g->cb_y - s->oy) / s->sy;
  return CPI_OK;
}

}  // namespace

extern "C" {

cpi_status cpi_lens_sampling_geometry(const cpi_geometry* g, const cpi_lens_sampling* s,
                                      cpi_geometry* out) {
  return guarded([&]() -> cpi_status {
    cpi::RefocusPlan pl;
    std::string why;
    cpi_status st = cpi::plan_refocus(g, 1, &pl, &why);
    if (st != CPI_OK) return set_error(st, why);
    cpi_geometry gs;
    st = lens_geometry(g, s, &gs);
    if (st != CPI_OK) return st;
    st = cpi::plan_refocus(&gs, 1, &pl, &why);
    if (st != CPI_OK) return set_error(st, "resampled views: " + why);
    if (!out) return set_error(CPI_ERR_INVALID_ARG, "out is null");
    *out = gs;
    return CPI_OK;
  });
}

cpi_status cpi_resample_views(const float* gamma, const cpi_geometry* g,
                              const cpi_lens_sampling* s, float* views, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi_geometry gs;
    cpi_status st = cpi_lens_sampling_geometry(g, s, &gs);
    if (st != CPI_OK) return st;
    if (!gamma || !views) return set_error(CPI_ERR_INVALID_ARG, "null device pointer");
    if (!aligned16(gamma) || !aligned16(views))
      return set_error(CPI_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
    hipStream_t sm = static_cast<hipStream_t>(stream);
    ProfScope ps("refocus_resample", sm);
    CPI_HIP(cpi::resample_views(gamma, int64_t(g->wa) * g->ha, g->wb, g->hb, s->nx, s->ny, s->ox,
                                s->oy, s->sx, s->sy, views, sm),
            "resample views");
    return CPI_OK;
  });
}

cpi_status cpi_refocus_resampled_workspace_size(const cpi_geometry* g, const cpi_lens_sampling* s,
                                                int32_t n_alpha, size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return set_error(CPI_ERR_INVALID_ARG, "bytes is null");
    cpi_geometry gs;
    cpi_status st = cpi_lens_sampling_geometry(g, s, &gs);
    if (st != CPI_OK) return st;
    cpi::RefocusPlan pl;
    std::string why;
    st = cpi::plan_refocus(&gs, n_alpha, &pl, &why);
    if (st != CPI_OK) return set_error(st, why);
    const size_t vb = (size_t(gs.wb) * gs.hb * size_t(g->wa) * g->ha * 4 + 255) / 256 * 256;
    *bytes = vb + pl.total;
    return CPI_OK;
  });
}

cpi_status cpi_refocus_resampled(const float* gamma, const cpi_geometry* g,
                                 const cpi_lens_sampling* s, const double* alphas,
                                 int32_t n_alpha, float* out, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  return guarded([&]() -> cpi_status {
    size_t need = 0;
    cpi_status st = cpi_refocus_resampled_workspace_size(g, s, n_alpha, &need);
    if (st != CPI_OK) return st;
    if (!workspace || !aligned16(workspace))
      return set_error(CPI_ERR_INVALID_ARG, "workspace must be a 16-byte aligned device pointer");
    if (workspace_bytes < need)
      return set_error(CPI_ERR_WORKSPACE,
                       "refocus workspace too small: need " + std::to_string(need) + " bytes");
    cpi_geometry gs;
    st = cpi_lens_sampling_geometry(g, s, &gs);
    if (st != CPI_OK) return st;
    std::string why;
    st = cpi::validate_alphas(&gs, alphas, n_alpha, &why);
    if (st != CPI_OK) return set_error(st, why);
    if (!out || !aligned16(out))
      return set_error(CPI_ERR_INVALID_ARG, "out must be a 16-byte aligned device pointer");
    float* views = static_cast<float*>(workspace);
    const size_t vb = (size_t(gs.wb) * gs.hb * size_t(g->wa) * g->ha * 4 + 255) / 256 * 256;
    st = cpi_resample_views(gamma, g, s, views, stream);
    if (st != CPI_OK) return st;
    return cpi::refocus_enqueue(views, &gs, alphas, n_alpha, out,
                                static_cast<uint8_t*>(workspace) + vb, workspace_bytes - vb,
                                static_cast<hipStream_t>(stream), nullptr, false);
  });
}

cpi_status cpi_measure_peaks_scratch_size(size_t copy_bytes, size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return set_error(CPI_ERR_INVALID_ARG, "bytes is null");
    if (copy_bytes == 0 || copy_bytes % 16)
      return set_error(CPI_ERR_INVALID_ARG, "copy_bytes must be a positive multiple of 16");
    *bytes = cpi::peaks_scratch_bytes(copy_bytes);
    return CPI_OK;
  });
}

cpi_status cpi_measure_peaks(void* scratch, size_t scratch_bytes, size_t copy_bytes,
                             double* int8_ops_per_s, double* fp4_ops_per_s,
                             double* copy_bytes_per_s, void* stream) {
  return guarded([&]() -> cpi_status {
    if (!scratch || !int8_ops_per_s || !fp4_ops_per_s || !copy_bytes_per_s)
      return set_error(CPI_ERR_INVALID_ARG, "null argument");
    if (copy_bytes == 0 || copy_bytes % 16)
      return set_error(CPI_ERR_INVALID_ARG, "copy_bytes must be a positive multiple of 16");
    if (!aligned16(scratch)) return set_error(CPI_ERR_INVALID_ARG, "scratch must be 16-byte aligned");
    if (scratch_bytes < cpi::peaks_scratch_bytes(copy_bytes))
      return set_error(CPI_ERR_WORKSPACE, "scratch smaller than cpi_measure_peaks_scratch_size");
    CPI_HIP(cpi::measure_peaks(static_cast<uint8_t*>(scratch), copy_bytes,
                               static_cast<hipStream_t>(stream), int8_ops_per_s, fp4_ops_per_s,
                               copy_bytes_per_s),
            "peaks");
    return CPI_OK;
  });
}

cpi_status cpi_set_mma_encoding(cpi_mma_encoding enc) {
  return guarded([&]() -> cpi_status {
    if (enc != CPI_MMA_AUTO && enc != CPI_MMA_INT8)
      return set_error(CPI_ERR_INVALID_ARG, "unknown matrix-core encoding");
    cpi::set_mma_encoding(int(enc));
    return CPI_OK;
  });
}

cpi_mma_encoding cpi_get_mma_encoding(void) {
  return cpi_mma_encoding(cpi::get_mma_encoding());
}

// ---------------------------------------------------------------------------
// Streaming
// ---------------------------------------------------------------------------

}  // extern "C"

struct cpi_stream_s {
  cpi::StreamPlan plan;
  int64_t pa = 0, pb = 0;
  int fmt = 0;
  uint8_t* ws = nullptr;
  hipStream_t st = nullptr;
  int64_t n_total = 0;
  // FP32 Gamma buffers: push k writes buffer k % gamma_buffers; `cur` is the
  // one the latest push (or checkpoint load) wrote.  written[b] is recorded
  // on st after a write of buffer b; read[b] on the refocus stream after an
  // asynchronous refocus of it, and the next write of b waits for it.
  int64_t writes = 0;
  int cur = 0;
  // false for the internal streams of blocked correlation: pushes then only
  // fold the sums (the outputs are made once, from the final state)
  bool refresh_gamma32 = true;
  hipEvent_t written[2] = {nullptr, nullptr};
  hipEvent_t read[2] = {nullptr, nullptr};
  bool read_pending[2] = {false, false};
  float* gamma32(int b) const {
    return reinterpret_cast<float*>(ws + (b == 0 ? plan.off_gamma32 : plan.off_gamma32b));
  }
  // Host chunks are copied on the device's copy stream (shared by the
  // handles, see make_copy_stream) into one of two staging pairs, so that the
  // copy of chunk k + 1 overlaps the work on chunk k: copied[b] is recorded
  // after the copy into pair b, staged_free[b] on st after the push that
  // read it.
  hipStream_t cst = nullptr;
  int stage_next = 0;
  hipEvent_t copied[2] = {nullptr, nullptr};
  hipEvent_t staged_free[2] = {nullptr, nullptr};
  bool stage_used[2] = {false, false};
  ~cpi_stream_s() {
    for (hipEvent_t e : {written[0], written[1], read[0], read[1], copied[0], copied[1],
                         staged_free[0], staged_free[1]})
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

constexpr uint64_t kStateMagic = 0x31415453495043ull;   // "CPISTA1"

struct StateHeader {
  uint64_t magic;
  int64_t pa, pb, fmt, n_total;
};

size_t state_bytes(const cpi_stream_s* s) {
  return sizeof(StateHeader) + size_t(s->pa) * 8 + size_t(s->pb) * 8 +
         size_t(s->pa) * size_t(s->pb) * (s->plan.state64 ? 8 : 4);
}

// The buffer the next Gamma32 write goes to; the stream waits until an
// asynchronous refocus of it has finished.
hipError_t gamma32_write_begin(cpi_stream_s* h, int* b) {
  *b = int(h->writes % h->plan.gamma_buffers);
  if (h->read_pending[*b]) {
    hipError_t e = hipStreamWaitEvent(h->st, h->read[*b], 0);
    if (e != hipSuccess) return e;
    h->read_pending[*b] = false;
  }
  return hipSuccess;
}

hipError_t gamma32_write_end(cpi_stream_s* h, int b) {
  h->cur = b;
  ++h->writes;
  return hipEventRecord(h->written[b], h->st);
}

cpi_status stream_push_device(cpi_stream_s* h, const uint8_t* fa, const uint8_t* fb, int64_t k) {
  if (k <= 0 || k > h->plan.max_chunk)
    return set_error(CPI_ERR_INVALID_ARG, "chunk size must be in [1, max_chunk]");
  const int64_t n_new = h->n_total + k;
  if (!cpi::overflow_ok(n_new, h->fmt))
    return set_error(CPI_ERR_OVERFLOW, "total frame count would break the exact bounds");
  if (h->fmt == CPI_FRAMES_BIT1 && n_new >= (int64_t(1) << 31))
    return set_error(CPI_ERR_OVERFLOW, "int32 stream state limited to 2^31 - 1 frames");
  cpi::CorrPlan cp;
  std::string why;
  cpi_status s = cpi::plan_correlate(k, h->pa, h->pb, h->fmt, &cp, &why);
  if (s != CPI_OK) return set_error(s, why);
  // The chunk plan uses this chunk's padding; offsets come from the
  // max-chunk plan, whose regions are at least as large.
  const cpi::CorrPlan& mp = h->plan.chunk;
  uint8_t* cws = h->ws + h->plan.off_chunk_ws;
  int64_t* csum_a = reinterpret_cast<int64_t*>(cws + mp.off_sum_a);
  int64_t* csum_b = reinterpret_cast<int64_t*>(cws + mp.off_sum_b);
  uint32_t* stats = reinterpret_cast<uint32_t*>(cws + mp.off_stats);
  uint8_t* op_a = cws + mp.off_op_a;
  uint8_t* op_b = cws + mp.off_op_b;
  int64_t* tot_a = reinterpret_cast<int64_t*>(h->ws + h->plan.off_sum_a);
  int64_t* tot_b = reinterpret_cast<int64_t*>(h->ws + h->plan.off_sum_b);
  hipStream_t st = h->st;
  {
    // chunk popcount sums, the 64 flag words and (byte frames) the byte sums
    cpi::ZeroRanges z;
    z.add(csum_a, cp.pa_pad);
    z.add(csum_b, cp.pb_pad);
    z.add(stats, 32);
    if (h->fmt != CPI_FRAMES_BIT1) {
      z.add(cws + mp.off_sum2_a, cp.pa_pad);
      z.add(cws + mp.off_sum2_b, cp.pb_pad);
    }
    CPI_HIP(cpi::zero_ranges(z, st), "fill");
  }

  cpi::GemmArgs g;
  g.opm = op_b;
  g.opn = op_a;
  g.m_pad = cp.pb_pad;
  g.n_pad = cp.pa_pad;
  g.layout = CPI_GAMMA_VIEW_MAJOR;
  g.pa = h->pa;
  g.pb = h->pb;
  g.n = n_new;
  g.kchunk = k;
  g.sum_a = tot_a;
  g.sum_b = tot_b;
  g.csum_a = csum_a;
  g.csum_b = csum_b;
  g.stats = stats;

  const bool fp4 = cpi::bits_use_fp4(cp.kpad_bits / cpi::kBitBlock);
  g.fp4 = fp4 ? 1 : 0;
  if (h->fmt == CPI_FRAMES_BIT1) {
    {
      ProfScope ps("ingest", st);
      // the chunk's popcounts are added straight into the running sums
      const cpi::IngestJob ja{fa, h->pa, cp.pa_pad, op_a, tot_a, nullptr, 0};
      const cpi::IngestJob jb{fb, h->pb, cp.pb_pad, op_b, tot_b, nullptr, fp4 ? 1 : 0};
      CPI_HIP(cpi::ingest_bits(ja, jb, k, cp.kpad_bits, st), "ingest");
    }
    int b = 0;
    if (h->refresh_gamma32) {
      CPI_HIP(gamma32_write_begin(h, &b), "gamma buffer");
      g.gamma_f32 = h->gamma32(b);
    }
    {
      ProfScope ps("gemm", st);
      g.row_bytes = cp.row_bytes_bits;
      g.kblocks = cp.kpad_bits / cpi::kBitBlock;
      g.mode = cpi::EPI_STREAM32;
      g.acc32 = reinterpret_cast<int32_t*>(h->ws + h->plan.off_sab);
      CPI_HIP(cpi::gemm_correlate(g, true, st), "gemm");
    }
    if (h->refresh_gamma32) CPI_HIP(gamma32_write_end(h, b), "gamma buffer");
  } else {
    int64_t* csum2_a = reinterpret_cast<int64_t*>(cws + mp.off_sum2_a);
    int64_t* csum2_b = reinterpret_cast<int64_t*>(cws + mp.off_sum2_b);
    {
      ProfScope ps("ingest", st);
      const cpi::IngestJob ja{fa, h->pa, cp.pa_pad, op_a, csum_a, csum2_a, 0};
      const cpi::IngestJob jb{fb, h->pb, cp.pb_pad, op_b, csum_b, csum2_b, fp4 ? 1 : 0};
      CPI_HIP(cpi::u8_to_bits(ja, jb, k, cp.kpad_bits, stats, st), "ingest");
      CPI_HIP(cpi::u8_sums(ja, jb, k, stats, st), "sums");
      CPI_HIP(cpi::add_select_i64(tot_a, csum_a, csum2_a, cp.pa_pad, stats, st), "sums");
      CPI_HIP(cpi::add_select_i64(tot_b, csum_b, csum2_b, cp.pb_pad, stats, st), "sums");
      CPI_HIP(cpi::u8_to_bytes(ja, jb, k, cp.kpad_bytes, stats, st), "ingest");
    }
    int b = 0;
    if (h->refresh_gamma32) {
      CPI_HIP(gamma32_write_begin(h, &b), "gamma buffer");
      g.gamma_f32 = h->gamma32(b);
    }
    ProfScope ps("gemm", st);
    g.mode = cpi::EPI_STREAM64;
    g.acc64 = reinterpret_cast<int64_t*>(h->ws + h->plan.off_sab);
    cpi::GemmArgs gb = g;
    gb.row_bytes = cp.row_bytes_bits;
    gb.kblocks = cp.kpad_bits / cpi::kBitBlock;
    gb.cond = 1;
    CPI_HIP(cpi::gemm_correlate(gb, true, st), "gemm");
    cpi::GemmArgs gy = g;
    gy.row_bytes = cp.row_bytes_bytes;
    gy.kblocks = cp.kpad_bytes / cpi::kByteBlock;
    gy.cond = 2;
    gy.offset_from_stats = 1;
    gy.csum_a = csum2_a;
    gy.csum_b = csum2_b;
    CPI_HIP(cpi::gemm_correlate(gy, false, st), "gemm");
    if (h->refresh_gamma32) CPI_HIP(gamma32_write_end(h, b), "gamma buffer");
  }
  h->n_total = n_new;
  return CPI_OK;
}

// The copy stream of the workspace's device: one per device for the
// process, made at first use and kept (each handle orders its copies with
// its own events).  Making a stream per handle would add hardware-queue
// users: with the runtime's default of four queues, streams then share them,
// and a refocus stream sharing a queue with the update stream loses its
// overlap.
std::mutex g_copy_mu;
hipStream_t g_copy_stream[64] = {};

hipError_t make_copy_stream(cpi_stream_s* h) {
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, h->ws);
  if (e != hipSuccess) return e;
  if (at.device < 0 || at.device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_copy_mu);
  if (!g_copy_stream[at.device]) {
    int cur_dev = 0;
    e = hipGetDevice(&cur_dev);
    if (e != hipSuccess) return e;
    e = hipSetDevice(at.device);
    if (e != hipSuccess) return e;
    e = hipStreamCreateWithFlags(&g_copy_stream[at.device], hipStreamNonBlocking);
    const hipError_t e2 = hipSetDevice(cur_dev);
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
  }
  h->cst = g_copy_stream[at.device];
  return hipSuccess;
}

cpi_status stream_create(int64_t pa, int64_t pb, cpi_frame_format fmt, int64_t max_chunk,
                         int gamma_buffers, void* workspace, size_t bytes, void* stream,
                         cpi_stream_t* out) {
  if (!out) return set_error(CPI_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  cpi::StreamPlan pl;
  std::string why;
  cpi_status s = cpi::plan_stream(pa, pb, int(fmt), max_chunk, &pl, &why, gamma_buffers);
  if (s != CPI_OK) return set_error(s, why);
  if (!workspace || !aligned16(workspace))
    return set_error(CPI_ERR_INVALID_ARG, "workspace must be a 16-byte aligned device pointer");
  if (bytes < pl.total)
    return set_error(CPI_ERR_WORKSPACE,
                     "stream workspace too small: need " + std::to_string(pl.total) + " bytes");
  std::unique_ptr<cpi_stream_s> h(new cpi_stream_s());
  h->plan = pl;
  h->pa = pa;
  h->pb = pb;
  h->fmt = int(fmt);
  h->ws = static_cast<uint8_t*>(workspace);
  h->st = static_cast<hipStream_t>(stream);
  h->refresh_gamma32 = gamma_buffers > 0;
  for (int b = 0; b < 2; ++b)
    for (hipEvent_t* e : {&h->written[b], &h->read[b], &h->copied[b], &h->staged_free[b]})
      CPI_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming), "stream init");
  const int64_t sab_words = pa * pb * (pl.state64 ? 2 : 1);
  CPI_HIP(cpi::fill_u32(reinterpret_cast<uint32_t*>(h->ws + pl.off_sab), sab_words, 0, h->st),
          "stream init");
  CPI_HIP(cpi::fill_u64(reinterpret_cast<uint64_t*>(h->ws + pl.off_sum_a), pl.chunk.pa_pad, 0,
                        h->st),
          "stream init");
  CPI_HIP(cpi::fill_u64(reinterpret_cast<uint64_t*>(h->ws + pl.off_sum_b), pl.chunk.pb_pad, 0,
                        h->st),
          "stream init");
  // made now rather than at the first host push, which would pay for it
  // (the internal handles of blocked correlation push device frames only)
  if (gamma_buffers > 0) CPI_HIP(make_copy_stream(h.get()), "stream init");
  *out = h.release();
  return CPI_OK;
}

}  // namespace

extern "C" {

cpi_status cpi_stream_workspace_size_ex(int64_t pa, int64_t pb, cpi_frame_format fmt,
                                        int64_t max_chunk, int32_t gamma_buffers,
                                        size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!bytes) return set_error(CPI_ERR_INVALID_ARG, "bytes is null");
    if (gamma_buffers != 1 && gamma_buffers != 2)
      return set_error(CPI_ERR_INVALID_ARG, "gamma_buffers must be 1 or 2");
    cpi::StreamPlan pl;
    std::string why;
    cpi_status s = cpi::plan_stream(pa, pb, int(fmt), max_chunk, &pl, &why, gamma_buffers);
    if (s != CPI_OK) return set_error(s, why);
    *bytes = pl.total;
    return CPI_OK;
  });
}

cpi_status cpi_stream_workspace_size(int64_t pa, int64_t pb, cpi_frame_format fmt,
                                     int64_t max_chunk, size_t* bytes) {
  return cpi_stream_workspace_size_ex(pa, pb, fmt, max_chunk, 1, bytes);
}

cpi_status cpi_stream_create_ex(int64_t pa, int64_t pb, cpi_frame_format fmt, int64_t max_chunk,
                                int32_t gamma_buffers, void* workspace, size_t bytes,
                                void* stream, cpi_stream_t* out) {
  return guarded([&]() -> cpi_status {
    if (gamma_buffers != 1 && gamma_buffers != 2)
      return set_error(CPI_ERR_INVALID_ARG, "gamma_buffers must be 1 or 2");
    return stream_create(pa, pb, fmt, max_chunk, gamma_buffers, workspace, bytes, stream, out);
  });
}

cpi_status cpi_stream_create(int64_t pa, int64_t pb, cpi_frame_format fmt, int64_t max_chunk,
                             void* workspace, size_t bytes, void* stream, cpi_stream_t* out) {
  return guarded([&]() -> cpi_status {
    return stream_create(pa, pb, fmt, max_chunk, 1, workspace, bytes, stream, out);
  });
}

cpi_status cpi_stream_push(cpi_stream_t s, const void* chunk_a, const void* chunk_b, int64_t k) {
  return guarded([&]() -> cpi_status {
    if (!s) return set_error(CPI_ERR_INVALID_ARG, "stream handle is null");
    cpi_status c = check_frames(chunk_a, chunk_b);
    if (c != CPI_OK) return c;
    return stream_push_device(s, static_cast<const uint8_t*>(chunk_a),
                              static_cast<const uint8_t*>(chunk_b), k);
  });
}

cpi_status cpi_stream_push_host(cpi_stream_t s, const void* chunk_a, const void* chunk_b,
                                int64_t k) {
  return guarded([&]() -> cpi_status {
    if (!s) return set_error(CPI_ERR_INVALID_ARG, "stream handle is null");
    if (!chunk_a || !chunk_b) return set_error(CPI_ERR_INVALID_ARG, "chunk pointers must not be null");
    if (k <= 0 || k > s->plan.max_chunk)
      return set_error(CPI_ERR_INVALID_ARG, "chunk size must be in [1, max_chunk]");
    if (!s->cst) CPI_HIP(make_copy_stream(s), "copy stream");
    const int sb = s->stage_next;
    uint8_t* da = s->ws + (sb == 0 ? s->plan.off_stage_a : s->plan.off_stage_a2);
    uint8_t* db = s->ws + (sb == 0 ? s->plan.off_stage_b : s->plan.off_stage_b2);
    const size_t ba = size_t(k) * size_t(cpi::frame_bytes(s->pa, s->fmt));
    const size_t bb = size_t(k) * size_t(cpi::frame_bytes(s->pb, s->fmt));
    if (s->stage_used[sb]) CPI_HIP(hipStreamWaitEvent(s->cst, s->staged_free[sb], 0), "copy chunk");
    CPI_HIP(hipMemcpyAsync(da, chunk_a, ba, hipMemcpyHostToDevice, s->cst), "copy chunk");
    CPI_HIP(hipMemcpyAsync(db, chunk_b, bb, hipMemcpyHostToDevice, s->cst), "copy chunk");
    CPI_HIP(hipEventRecord(s->copied[sb], s->cst), "copy chunk");
    CPI_HIP(hipStreamWaitEvent(s->st, s->copied[sb], 0), "copy chunk");
    s->stage_next ^= 1;
    const cpi_status c = stream_push_device(s, da, db, k);
    CPI_HIP(hipEventRecord(s->staged_free[sb], s->st), "copy chunk");
    s->stage_used[sb] = true;
    return c;
  });
}

cpi_status cpi_stream_frames(cpi_stream_t s, int64_t* n) {
  return guarded([&]() -> cpi_status {
    if (!s || !n) return set_error(CPI_ERR_INVALID_ARG, "null argument");
    *n = s->n_total;
    return CPI_OK;
  });
}

cpi_status cpi_stream_gamma(cpi_stream_t s, cpi_gamma_layout layout, double* gamma,
                            float* gamma_f32, int64_t* numer, int64_t* sum_a, int64_t* sum_b) {
  return guarded([&]() -> cpi_status {
    if (!s) return set_error(CPI_ERR_INVALID_ARG, "stream handle is null");
    if (layout != CPI_GAMMA_VIEW_MAJOR && layout != CPI_GAMMA_PIXEL_MAJOR)
      return set_error(CPI_ERR_INVALID_ARG, "unknown Gamma layout");
    const void* outs[5] = {gamma, gamma_f32, numer, sum_a, sum_b};
    for (const void* o : outs)
      if (o && !aligned16(o)) return set_error(CPI_ERR_INVALID_ARG, "outputs must be 16-byte aligned");
    if (s->n_total == 0) return set_error(CPI_ERR_NOT_READY, "no frames pushed yet");
    const int64_t* ta = reinterpret_cast<const int64_t*>(s->ws + s->plan.off_sum_a);
    const int64_t* tb = reinterpret_cast<const int64_t*>(s->ws + s->plan.off_sum_b);
    ProfScope ps("state_gamma", s->st);
    if (gamma || gamma_f32 || numer)
      CPI_HIP(cpi::state_gamma(s->ws + s->plan.off_sab, s->plan.state64, ta, tb, s->n_total, s->pa,
                               s->pb, int(layout), gamma, gamma_f32, numer, s->st),
              "stream gamma");
    if (sum_a)
      CPI_HIP(hipMemcpyAsync(sum_a, ta, size_t(s->pa) * 8, hipMemcpyDeviceToDevice, s->st), "copy sums");
    if (sum_b)
      CPI_HIP(hipMemcpyAsync(sum_b, tb, size_t(s->pb) * 8, hipMemcpyDeviceToDevice, s->st), "copy sums");
    return CPI_OK;
  });
}

cpi_status cpi_stream_gamma_f32_ptr(cpi_stream_t s, const float** gamma_f32) {
  return guarded([&]() -> cpi_status {
    if (!s || !gamma_f32) return set_error(CPI_ERR_INVALID_ARG, "null argument");
    *gamma_f32 = s->gamma32(s->cur);
    return CPI_OK;
  });
}

cpi_status cpi_stream_refocus(cpi_stream_t s, const cpi_geometry* g, const double* alphas,
                              int32_t n_alpha, float* out, void* workspace,
                              size_t workspace_bytes) {
  return guarded([&]() -> cpi_status {
    if (!s) return set_error(CPI_ERR_INVALID_ARG, "stream handle is null");
    if (s->n_total == 0) return set_error(CPI_ERR_NOT_READY, "no frames pushed yet");
    if (g && (int64_t(g->wa) * g->ha != s->pa || int64_t(g->wb) * g->hb != s->pb))
      return set_error(CPI_ERR_INVALID_ARG, "geometry does not match the stream's detectors");
    return cpi::refocus_enqueue(s->gamma32(s->cur), g, alphas, n_alpha, out, workspace,
                                workspace_bytes, s->st, nullptr, false);
  });
}

cpi_status cpi_stream_refocus_async(cpi_stream_t s, const cpi_geometry* g, const double* alphas,
                                    int32_t n_alpha, float* out, void* workspace,
                                    size_t workspace_bytes, void* refocus_stream) {
  return guarded([&]() -> cpi_status {
    if (!s) return set_error(CPI_ERR_INVALID_ARG, "stream handle is null");
    if (s->n_total == 0) return set_error(CPI_ERR_NOT_READY, "no frames pushed yet");
    if (g && (int64_t(g->wa) * g->ha != s->pa || int64_t(g->wb) * g->hb != s->pb))
      return set_error(CPI_ERR_INVALID_ARG, "geometry does not match the stream's detectors");
    hipStream_t rs = static_cast<hipStream_t>(refocus_stream);
    const int b = s->cur;
    CPI_HIP(hipStreamWaitEvent(rs, s->written[b], 0), "refocus wait");
    cpi_status st = cpi::refocus_enqueue(s->gamma32(b), g, alphas, n_alpha, out, workspace,
                                         workspace_bytes, rs, nullptr, false);
    if (st != CPI_OK) return st;
    CPI_HIP(hipEventRecord(s->read[b], rs), "refocus record");
    s->read_pending[b] = true;
    return CPI_OK;
  });
}

cpi_status cpi_stream_state_size(cpi_stream_t s, size_t* bytes) {
  return guarded([&]() -> cpi_status {
    if (!s || !bytes) return set_error(CPI_ERR_INVALID_ARG, "null argument");
    *bytes = state_bytes(s);
    return CPI_OK;
  });
}

cpi_status cpi_stream_save(cpi_stream_t s, void* host_buf, size_t bytes) {
  return guarded([&]() -> cpi_status {
    if (!s || !host_buf) return set_error(CPI_ERR_INVALID_ARG, "null argument");
    if (bytes < state_bytes(s)) return set_error(CPI_ERR_INVALID_ARG, "state buffer too small");
    uint8_t* dst = static_cast<uint8_t*>(host_buf);
    StateHeader hd{kStateMagic, s->pa, s->pb, s->fmt, s->n_total};
    std::memcpy(dst, &hd, sizeof(hd));
    size_t off = sizeof(hd);
    CPI_HIP(hipMemcpyAsync(dst + off, s->ws + s->plan.off_sum_a, size_t(s->pa) * 8,
                           hipMemcpyDeviceToHost, s->st), "save");
    off += size_t(s->pa) * 8;
    CPI_HIP(hipMemcpyAsync(dst + off, s->ws + s->plan.off_sum_b, size_t(s->pb) * 8,
                           hipMemcpyDeviceToHost, s->st), "save");
    off += size_t(s->pb) * 8;
    CPI_HIP(hipMemcpyAsync(dst + off, s->ws + s->plan.off_sab,
                           size_t(s->pa) * size_t(s->pb) * (s->plan.state64 ? 8 : 4),
                           hipMemcpyDeviceToHost, s->st), "save");
    CPI_HIP(hipStreamSynchronize(s->st), "save");
    return CPI_OK;
  });
}

cpi_status cpi_stream_load(cpi_stream_t s, const void* host_buf, size_t bytes) {
  return guarded([&]() -> cpi_status {
    if (!s || !host_buf) return set_error(CPI_ERR_INVALID_ARG, "null argument");
    if (bytes < state_bytes(s)) return set_error(CPI_ERR_INVALID_ARG, "state buffer too small");
    const uint8_t* src = static_cast<const uint8_t*>(host_buf);
    StateHeader hd;
    std::memcpy(&hd, src, sizeof(hd));
    if (hd.magic != kStateMagic || hd.pa != s->pa || hd.pb != s->pb || hd.fmt != s->fmt ||
        hd.n_total < 0 || (hd.n_total > 0 && !cpi::overflow_ok(hd.n_total, s->fmt)))
      return set_error(CPI_ERR_INVALID_ARG, "checkpoint does not match this stream");
    size_t off = sizeof(hd);
    CPI_HIP(hipMemcpyAsync(s->ws + s->plan.off_sum_a, src + off, size_t(s->pa) * 8,
                           hipMemcpyHostToDevice, s->st), "load");
    off += size_t(s->pa) * 8;
    CPI_HIP(hipMemcpyAsync(s->ws + s->plan.off_sum_b, src + off, size_t(s->pb) * 8,
                           hipMemcpyHostToDevice, s->st), "load");
    off += size_t(s->pb) * 8;
    CPI_HIP(hipMemcpyAsync(s->ws + s->plan.off_sab, src + off,
                           size_t(s->pa) * size_t(s->pb) * (s->plan.state64 ? 8 : 4),
                           hipMemcpyHostToDevice, s->st), "load");
    s->n_total = hd.n_total;
    if (s->n_total > 0) {
      const int64_t* ta = reinterpret_cast<const int64_t*>(s->ws + s->plan.off_sum_a);
      const int64_t* tb = reinterpret_cast<const int64_t*>(s->ws + s->plan.off_sum_b);
      int b = 0;
      CPI_HIP(gamma32_write_begin(s, &b), "load");
      CPI_HIP(cpi::state_gamma(s->ws + s->plan.off_sab, s->plan.state64, ta, tb, s->n_total, s->pa,
                               s->pb, CPI_GAMMA_VIEW_MAJOR, nullptr, s->gamma32(b), nullptr,
                               s->st),
              "load");
      CPI_HIP(gamma32_write_end(s, b), "load");
    }
    CPI_HIP(hipStreamSynchronize(s->st), "load");
    return CPI_OK;
  });
}

cpi_status cpi_profile_begin(void) {
  return guarded([&]() -> cpi_status {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_on = true;
    return CPI_OK;
  });
}

cpi_status cpi_profile_end(void) {
  return guarded([&]() -> cpi_status {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = false;
    return CPI_OK;
  });
}

cpi_status cpi_profile_query(const char* group, int64_t* launches, double* total_ms) {
  return guarded([&]() -> cpi_status {
    if (!group || !launches || !total_ms) return set_error(CPI_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int64_t cnt = 0;
    double tot = 0.0;
    for (ProfRec& r : g_prof) {
      if (r.group != group) continue;
      CPI_HIP(hipEventSynchronize(r.b), "profile");
      float ms = 0.f;
      CPI_HIP(hipEventElapsedTime(&ms, r.a, r.b), "profile");
      ++cnt;
      tot += ms;
    }
    *launches = cnt;
    *total_ms = tot;
    return CPI_OK;
  });
}

cpi_status cpi_stream_destroy(cpi_stream_t s) {
  return guarded([&]() -> cpi_status {
    delete s;
    return CPI_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Raw side-by-side sensor frames and frame files
// ---------------------------------------------------------------------------
namespace {

cpi_status check_sidebyside(const cpi_sidebyside* f) {
  if (!f) return set_error(CPI_ERR_INVALID_ARG, "frame layout is null");
  if (f->frame_w <= 0 || f->frame_h <= 0 || (f->frame_w & 1))
    return set_error(CPI_ERR_INVALID_ARG, "frame_w must be positive and even, frame_h positive");
  if (f->roi_w <= 0 || f->roi_h <= 0 || f->roi_x < 0 || f->roi_y < 0 ||
      int64_t(f->roi_x) + f->roi_w > f->frame_w / 2 || int64_t(f->roi_y) + f->roi_h > f->frame_h)
    return set_error(CPI_ERR_INVALID_ARG, "region of interest outside the half frame");
  return CPI_OK;
}

int64_t raw_frame_bytes(const cpi_sidebyside* f) {
  return (int64_t(f->frame_w) * f->frame_h + 7) / 8;
}

// Whole frames in a file; a size that is not a multiple of the frame is an error.
cpi_status file_frames(const char* path, int64_t fbytes, int64_t* frames) {
  if (!path) return set_error(CPI_ERR_INVALID_ARG, "file path is null");
  std::FILE* fp = std::fopen(path, "rb");
  if (!fp) return set_error(CPI_ERR_INVALID_ARG, std::string("cannot open ") + path);
  const bool ok = fseeko(fp, 0, SEEK_END) == 0;
  const off_t size = ok ? ftello(fp) : off_t(-1);
  std::fclose(fp);
  if (size < 0) return set_error(CPI_ERR_INVALID_ARG, std::string("cannot size ") + path);
  if (size % fbytes != 0)
    return set_error(CPI_ERR_INVALID_ARG,
                     std::string(path) + " does not hold a whole number of frames");
  *frames = int64_t(size) / fbytes;
  return CPI_OK;
}

// Events and the open file of one ingest call, released on every exit path.
struct IngestResources {
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::FILE* fp = nullptr;
  ~IngestResources() {
    for (hipEvent_t e : ev)
      if (e) hipEventDestroy(e);
    if (fp) std::fclose(fp);
  }
};

}  // namespace

extern "C" {

cpi_status cpi_split_sidebyside(const void* frames, int64_t n, const cpi_sidebyside* f,
                                void* frames_a, void* frames_b, void* stream) {
  return guarded([&]() -> cpi_status {
    cpi_status c = check_sidebyside(f);
    if (c != CPI_OK) return c;
    if (!frames || !frames_a || !frames_b)
      return set_error(CPI_ERR_INVALID_ARG, "frame pointers must not be null");
    if (n <= 0) return set_error(CPI_ERR_INVALID_ARG, "n must be positive");
    CPI_HIP(cpi::split_sidebyside(static_cast<const uint8_t*>(frames), n, f->frame_w, f->frame_h,
                                  f->roi_x, f->roi_y, f->roi_w, f->roi_h,
                                  static_cast<uint8_t*>(frames_a), static_cast<uint8_t*>(frames_b),
                                  static_cast<hipStream_t>(stream)),
            "split");
    return CPI_OK;
  });
}

cpi_status cpi_file_frames(const char* path, const cpi_sidebyside* f, int64_t* frames) {
  return guarded([&]() -> cpi_status {
    cpi_status c = check_sidebyside(f);
    if (c != CPI_OK) return c;
    if (!frames) return set_error(CPI_ERR_INVALID_ARG, "frames is null");
    return file_frames(path, raw_frame_bytes(f), frames);
  });
}

cpi_status cpi_stream_ingest_files(cpi_stream_t s, const char* const* paths, int32_t n_paths,
                                   const cpi_sidebyside* f, void* host_a, void* host_b,
                                   size_t host_bytes, void* dev_raw, size_t dev_bytes,
                                   int64_t* frames) {
  return guarded([&]() -> cpi_status {
    if (!s) return set_error(CPI_ERR_INVALID_ARG, "stream handle is null");
    if (!paths || n_paths < 1 || !host_a || !host_b || !dev_raw || !frames)
      return set_error(CPI_ERR_INVALID_ARG, "null argument or no files");
    *frames = 0;
    cpi_status c = check_sidebyside(f);
    if (c != CPI_OK) return c;
    const int64_t roi_px = int64_t(f->roi_w) * f->roi_h;
    if (s->fmt != CPI_FRAMES_BIT1 || s->pa != roi_px || s->pb != roi_px)
      return set_error(CPI_ERR_INVALID_ARG,
                       "stream must hold 1-bit frames of roi_w*roi_h pixels on both detectors");
    const int64_t fb = raw_frame_bytes(f);
    int64_t piece = s->plan.max_chunk;
    piece = std::min<int64_t>(piece, int64_t(host_bytes) / fb);
    piece = std::min<int64_t>(piece, int64_t(dev_bytes) / fb);
    if (piece < 1) return set_error(CPI_ERR_INVALID_ARG, "buffers smaller than one raw frame");
    std::vector<int64_t> nf(size_t(n_paths), 0);
    for (int32_t i = 0; i < n_paths; ++i) {
      c = file_frames(paths[i], fb, &nf[size_t(i)]);
      if (c != CPI_OK) return c;
    }
    IngestResources res;
    for (hipEvent_t& e : res.ev)
      CPI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    uint8_t* host[2] = {static_cast<uint8_t*>(host_a), static_cast<uint8_t*>(host_b)};
    bool in_flight[2] = {false, false};
    uint8_t* raw = static_cast<uint8_t*>(dev_raw);
    uint8_t* sa = s->ws + s->plan.off_stage_a;
    uint8_t* sb = s->ws + s->plan.off_stage_b;
    int32_t file = -1;
    int64_t left = 0;
    // Reads the next piece (within one file) into buf; k = 0 when all are read.
    auto read_piece = [&](uint8_t* buf, int64_t* k) -> cpi_status {
      *k = 0;
      while (left == 0) {
        if (res.fp) {
          std::fclose(res.fp);
          res.fp = nullptr;
        }
        if (++file >= n_paths) return CPI_OK;
        left = nf[size_t(file)];
        if (left > 0) {
          res.fp = std::fopen(paths[file], "rb");
          if (!res.fp) return set_error(CPI_ERR_INVALID_ARG, std::string("cannot open ") + paths[file]);
        }
      }
      const int64_t want = std::min(left, piece);
      if (std::fread(buf, size_t(fb), size_t(want), res.fp) != size_t(want))
        return set_error(CPI_ERR_INVALID_ARG, std::string("short read from ") + paths[file]);
      left -= want;
      *k = want;
      return CPI_OK;
    };
    int slot = 0;
    int64_t k = 0;
    c = read_piece(host[0], &k);
    if (c != CPI_OK) return c;
    while (k > 0) {
      CPI_HIP(hipMemcpyAsync(raw, host[slot], size_t(k * fb), hipMemcpyHostToDevice, s->st),
              "copy frames");
      CPI_HIP(hipEventRecord(res.ev[slot], s->st), "event");
      in_flight[slot] = true;
      CPI_HIP(cpi::split_sidebyside(raw, k, f->frame_w, f->frame_h, f->roi_x, f->roi_y, f->roi_w,
                                    f->roi_h, sa, sb, s->st),
              "split");
      c = stream_push_device(s, sa, sb, k);
      if (c != CPI_OK) return c;
      *frames += k;
      // the other buffer is free once its last copy to the device has completed
      const int other = slot ^ 1;
      if (in_flight[other]) CPI_HIP(hipEventSynchronize(res.ev[other]), "event");
      in_flight[other] = false;
      c = read_piece(host[other], &k);
      if (c != CPI_OK) return c;
      slot = other;
    }
    return CPI_OK;
  });
}

}  // extern "C"
