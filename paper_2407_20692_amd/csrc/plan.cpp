// Host-side planning for the CPI library (no HIP dependencies).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace cpi {

namespace {

constexpr int64_t kMaxPix = int64_t(1) << 28;
constexpr int64_t kMaxPairs = int64_t(1) << 40;   // Pa * Pb
constexpr int64_t kMaxDim = 1 << 16;
constexpr double kMaxCoord = 1073741824.0;        // 2^30: coordinates stay int32

cpi_status fail(std::string* why, cpi_status s, const char* msg) {
  if (why) *why = msg;
  return s;
}

bool finite(double x) { return std::isfinite(x); }

}  // namespace

int64_t frame_bytes(int64_t npix, int fmt) {
  if (fmt == CPI_FRAMES_U8) return npix;
  if (fmt == CPI_FRAMES_BIT1) return (npix + 7) / 8;
  return -1;
}

bool overflow_ok(int64_t n, int fmt) {
  if (n <= 0) return false;
  // n*n < 2^53  <=>  n < 94906266 (94906265^2 < 2^53 < 94906266^2)
  if (n > 94906265) return false;
  const unsigned __int128 nn = (unsigned __int128)n * (unsigned __int128)n;
  const unsigned __int128 v = (fmt == CPI_FRAMES_U8) ? 255u : 1u;
  const unsigned __int128 lim = (unsigned __int128)1 << 63;
  return nn * v * v < lim;
}

cpi_status plan_correlate(int64_t n, int64_t pa, int64_t pb, int fmt, CorrPlan* p,
                          std::string* why) {
  if (!p) return fail(why, CPI_ERR_INVALID_ARG, "plan output is null");
  if (fmt != CPI_FRAMES_U8 && fmt != CPI_FRAMES_BIT1)
    return fail(why, CPI_ERR_INVALID_ARG, "unknown frame format");
  if (n <= 0) return fail(why, CPI_ERR_INVALID_ARG, "n must be positive");
  if (pa <= 0 || pb <= 0) return fail(why, CPI_ERR_INVALID_ARG, "pa and pb must be positive");
  if (pa > kMaxPix || pb > kMaxPix || pa * pb > kMaxPairs)
    return fail(why, CPI_ERR_INVALID_ARG, "pa * pb too large");
  if (!overflow_ok(n, fmt))
    return fail(why, CPI_ERR_OVERFLOW,
                "n^2 * max^2 must stay below 2^63 and n^2 below 2^53 (max = 255 for U8, 1 for BIT1)");
  CorrPlan q;
  q.n = n;
  q.pa = pa;
  q.pb = pb;
  q.fmt = fmt;
  q.pa_pad = round_up(pa, kRowPad);
  q.pb_pad = round_up(pb, kRowPad);
  q.kpad_bits = round_up(n, kBitBlock);
  q.row_bytes_bits = q.kpad_bits / 8;
  int64_t row = q.row_bytes_bits;
  if (fmt == CPI_FRAMES_U8) {
    q.kpad_bytes = round_up(n, kByteBlock);
    q.row_bytes_bytes = q.kpad_bytes;
    q.passes = int((n + kByteChunk - 1) / kByteChunk);
    if (q.row_bytes_bytes > row) row = q.row_bytes_bytes;
  }
  size_t off = 0;
  q.off_sum_a = off;
  off = align256(off + size_t(q.pa_pad) * 8);
  q.off_sum_b = off;
  off = align256(off + size_t(q.pb_pad) * 8);
  q.off_sum2_a = off;
  if (fmt == CPI_FRAMES_U8) off = align256(off + size_t(q.pa_pad) * 8);
  q.off_sum2_b = off;
  if (fmt == CPI_FRAMES_U8) off = align256(off + size_t(q.pb_pad) * 8);
  q.off_stats = off;
  off = align256(off + 256);
  q.off_op_a = off;
  off = align256(off + size_t(q.pa_pad) * size_t(row));
  q.off_op_b = off;
  off = align256(off + size_t(q.pb_pad) * size_t(row));
  q.off_acc64 = off;
  if (fmt == CPI_FRAMES_U8 && q.passes > 1) off = align256(off + size_t(pa) * size_t(pb) * 8);
  q.total = off;
  *p = q;
  return CPI_OK;
}

cpi_status plan_correlate_plain(int64_t n, int64_t pa, int64_t pb, int fmt,
                                PlainPlan* p, std::string* why) {
  if (!p) return fail(why, CPI_ERR_INVALID_ARG, "plan output is null");
  if (fmt != CPI_FRAMES_U8 && fmt != CPI_FRAMES_BIT1)
    return fail(why, CPI_ERR_INVALID_ARG, "unknown frame format");
  if (n <= 0) return fail(why, CPI_ERR_INVALID_ARG, "n must be positive");
  if (pa <= 0 || pb <= 0) return fail(why, CPI_ERR_INVALID_ARG, "pa and pb must be positive");
  if (pa > kMaxPix || pb > kMaxPix || pa * pb > kMaxPairs)
    return fail(why, CPI_ERR_INVALID_ARG, "pa * pb too large");
  if (n > (int64_t(1) << 31)) return fail(why, CPI_ERR_OVERFLOW, "n too large for the FP32 path");
  PlainPlan q;
  q.n = n;
  q.pa = pa;
  q.pb = pb;
  q.fmt = fmt;
  q.kpad = round_up(n, 16);
  q.pa_pad = round_up(pa, 128);
  q.pb_pad = round_up(pb, 128);
  size_t off = 0;
  q.off_fa = off;
  off = align256(off + size_t(q.kpad) * size_t(q.pa_pad) * 4);
  q.off_fb = off;
  off = align256(off + size_t(q.kpad) * size_t(q.pb_pad) * 4);
  q.off_sa = off;
  off = align256(off + size_t(q.pa_pad) * 4);
  q.off_sb = off;
  off = align256(off + size_t(q.pb_pad) * 4);
  q.total = off;
  *p = q;
  return CPI_OK;
}

cpi_status validate_geometry(const cpi_geometry* g, std::string* why) {
  if (!g) return fail(why, CPI_ERR_INVALID_ARG, "geometry is null");
  if (g->wa <= 0 || g->ha <= 0 || g->wb <= 0 || g->hb <= 0 || g->out_w <= 0 || g->out_h <= 0)
    return fail(why, CPI_ERR_INVALID_ARG, "geometry sizes must be positive");
  if (g->wa > kMaxDim || g->ha > kMaxDim || g->wb > kMaxDim || g->hb > kMaxDim ||
      g->out_w > kMaxDim || g->out_h > kMaxDim)
    return fail(why, CPI_ERR_INVALID_ARG, "geometry size above 65536");
  const int64_t pa = int64_t(g->wa) * g->ha, pb = int64_t(g->wb) * g->hb;
  if (pa > kMaxPix || pb > kMaxPix || pa * pb > kMaxPairs)
    return fail(why, CPI_ERR_INVALID_ARG, "Gamma too large");
  const double v[6] = {g->mag_x, g->mag_y, g->ca_x, g->ca_y, g->cb_x, g->cb_y};
  for (double x : v)
    if (!finite(x) || std::fabs(x) > 1048576.0)
      return fail(why, CPI_ERR_INVALID_ARG, "geometry parameters must be finite and below 2^20");
  return CPI_OK;
}

cpi_status validate_alphas(const cpi_geometry* g, const double* alphas, int32_t n_alpha,
                           std::string* why) {
  if (!alphas) return fail(why, CPI_ERR_INVALID_ARG, "alphas is null");
  if (n_alpha < 1 || n_alpha > kMaxAlpha)
    return fail(why, CPI_ERR_INVALID_ARG, "n_alpha must be in [1, 4096]");
  const double ax = std::fmax(std::fabs(g->ca_x), std::fabs(g->out_w - 1 - g->ca_x));
  const double ay = std::fmax(std::fabs(g->ca_y), std::fabs(g->out_h - 1 - g->ca_y));
  const double bx = std::fmax(std::fabs(g->cb_x), std::fabs(g->wb - 1 - g->cb_x));
  const double by = std::fmax(std::fabs(g->cb_y), std::fabs(g->hb - 1 - g->cb_y));
  for (int32_t k = 0; k < n_alpha; ++k) {
    const double a = alphas[k];
    if (!finite(a)) return fail(why, CPI_ERR_INVALID_ARG, "alpha values must be finite");
    const double cx = std::fabs(a) * ax + std::fabs(g->ca_x) + 2.0;
    const double cy = std::fabs(a) * ay + std::fabs(g->ca_y) + 2.0;
    const double sx = std::fabs(1.0 - a) * std::fabs(g->mag_x) * bx + 2.0;
    const double sy = std::fabs(1.0 - a) * std::fabs(g->mag_y) * by + 2.0;
    if (cx > kMaxCoord || cy > kMaxCoord || sx > kMaxCoord || sy > kMaxCoord)
      return fail(why, CPI_ERR_INVALID_ARG, "alpha gives interpolation coordinates beyond 2^30");
  }
  return CPI_OK;
}

cpi_status plan_refocus(const cpi_geometry* g, int32_t n_alpha, RefocusPlan* p,
                        std::string* why) {
  cpi_status s = validate_geometry(g, why);
  if (s != CPI_OK) return s;
  if (n_alpha < 1 || n_alpha > kMaxAlpha)
    return fail(why, CPI_ERR_INVALID_ARG, "n_alpha must be in [1, 4096]");
  if (!p) return fail(why, CPI_ERR_INVALID_ARG, "plan output is null");
  RefocusPlan q;
  q.table_stride = int64_t(g->out_w) + g->out_h + g->wb + g->hb;
  size_t off = 0;
  q.off_itab = off;
  off = align256(off + size_t(n_alpha) * size_t(q.table_stride) * 4);
  q.off_ftab = off;
  off = align256(off + size_t(n_alpha) * size_t(q.table_stride) * 4);
  q.off_ytab = off;
  off = align256(off + size_t(n_alpha) * size_t(g->hb) * size_t(g->out_h) * 16);
  // window bounds of the batched kernels: at most n_alpha plane groups (one
  // plane per work-group), ceil(out_w/64) tile columns and ceil(out_h/8) tile
  // rows
  q.off_bounds = off;
  const size_t groups = size_t(n_alpha);
  off = align256(off + groups * (size_t((g->out_w + 63) / 64) * size_t(g->wb) +
                                 size_t((g->out_h + 7) / 8) * size_t(g->hb)) * 8);
  q.off_partial = off;
  const int64_t splits = std::min<int64_t>(kMaxViewSplits, g->hb);
  q.partial_bytes = size_t(splits) * size_t(n_alpha) * size_t(g->out_w) * size_t(g->out_h) * 4;
  // Row-lane kernel: T (hb x ha x output columns per plane) of one chunk of
  // planes shares the partial-sum region.  Every chunk streams all of Gamma
  // once, so chunks are large: multiples of 16 planes, at most 256, as many
  // as fit max(partial sums, 4 GiB), and at least 16 while T of 16 planes
  // stays within 4 GiB.
  q.rows_wout_cap = round_up(g->out_w, 64);
  const size_t t_plane = size_t(g->hb) * size_t(g->ha) * size_t(q.rows_wout_cap) * 4;
  const size_t budget = std::max<size_t>(q.partial_bytes, size_t(4) << 30);
  int64_t chunk = std::min<int64_t>(round_up(n_alpha, 16), 256);
  while (chunk > 16 && size_t(chunk) * t_plane > budget) chunk -= 16;
  if (size_t(chunk) * t_plane > (size_t(4) << 30)) chunk = 0;
  q.rows_chunk = chunk;
  q.partial_bytes = std::max(q.partial_bytes, size_t(chunk) * t_plane);
  off = align256(off + q.partial_bytes);
  // per-view tables of one chunk: 3 words per (plane, output column, view
  // column) and a 4-word header per 64 or more pairs; touched-row ranges (at
  // most one per plane and lens-plane row)
  const size_t pairs = size_t(chunk) * size_t(q.rows_wout_cap) * size_t(g->wb);
  q.off_rows_xe = off;
  off = align256(off + pairs * 12 + pairs / 4 + 16);
  q.off_rows_yr = off;
  off = align256(off + size_t(chunk) * size_t(g->hb) * 8 + 8);
  q.total = off;
  *p = q;
  return CPI_OK;
}

cpi_status plan_stream(int64_t pa, int64_t pb, int fmt, int64_t max_chunk, StreamPlan* p,
                       std::string* why, int gamma_buffers) {
  if (!p) return fail(why, CPI_ERR_INVALID_ARG, "plan output is null");
  if (max_chunk <= 0) return fail(why, CPI_ERR_INVALID_ARG, "max_chunk must be positive");
  if (gamma_buffers < 0 || gamma_buffers > 2)
    return fail(why, CPI_ERR_INVALID_ARG, "gamma_buffers must be 1 or 2");
  if (fmt == CPI_FRAMES_U8 && max_chunk > kByteChunk)
    return fail(why, CPI_ERR_INVALID_ARG, "U8 chunks are limited to 131008 frames");
  if (max_chunk > kMaxPassFrames)
    return fail(why, CPI_ERR_INVALID_ARG, "chunks are limited to 16776704 frames");
  StreamPlan q;
  cpi_status s = plan_correlate(max_chunk, pa, pb, fmt, &q.chunk, why);
  if (s != CPI_OK) return s;
  q.max_chunk = max_chunk;
  q.state64 = (fmt == CPI_FRAMES_U8);
  size_t off = 0;
  q.off_chunk_ws = off;
  off = align256(off + q.chunk.total);
  q.off_sab = off;
  off = align256(off + size_t(pa) * size_t(pb) * (q.state64 ? 8 : 4));
  q.off_sum_a = off;
  off = align256(off + size_t(q.chunk.pa_pad) * 8);
  q.off_sum_b = off;
  off = align256(off + size_t(q.chunk.pb_pad) * 8);
  q.off_gamma32 = off;   // (no buffer when gamma_buffers is 0: sums only)
  off = align256(off + (gamma_buffers > 0 ? size_t(pa) * size_t(pb) * 4 : 0));
  q.off_stage_a = off;
  off = align256(off + size_t(max_chunk) * size_t(frame_bytes(pa, fmt)));
  q.off_stage_b = off;
  off = align256(off + size_t(max_chunk) * size_t(frame_bytes(pb, fmt)));
  q.off_stage_a2 = off;
  off = align256(off + size_t(max_chunk) * size_t(frame_bytes(pa, fmt)));
  q.off_stage_b2 = off;
  off = align256(off + size_t(max_chunk) * size_t(frame_bytes(pb, fmt)));
  q.gamma_buffers = gamma_buffers;
  q.off_gamma32b = q.off_gamma32;
  if (gamma_buffers == 2) {
    q.off_gamma32b = off;
    off = align256(off + size_t(pa) * size_t(pb) * 4);
  }
  q.total = off;
  *p = q;
  return CPI_OK;
}

}  // namespace cpi
