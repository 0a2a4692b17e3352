// Host-side planning for the CPI library: argument validation, overflow
// bounds, operand padding and workspace layouts.  Free of HIP so that it
// can be built and tested with a plain host compiler.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "cpi.h"

namespace cpi {

// Operand rows (pixels of either detector) are padded to a whole number of
// GEMM work-group tiles; frames (the contraction dimension) to whole blocks.
constexpr int64_t kRowPad = 256;
constexpr int64_t kBitBlock = 512;      // frames per 64-byte row segment, 1 bit/frame
constexpr int64_t kByteBlock = 64;      // frames per 64-byte row segment, 1 byte/frame
// Frames per int32 pass for byte operands: 131008 * 128 * 128 < 2^31 - 1.
constexpr int64_t kByteChunk = 131008;
// Frames one pass of the bit-row ingest takes (row offsets within a tile of
// 1024 rows stay below 2^31 bytes).
constexpr int64_t kMaxPassFrames = (int64_t(1) << 24) - kBitBlock;
constexpr int kMaxAlpha = 4096;
constexpr int kAlphaPerLaunch = 64;     // plane parameters passed by value per table launch

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of one frame in the given format (-1 for an unknown format).
int64_t frame_bytes(int64_t npix, int fmt);

// Int64 / FP64 bounds of the exact evaluation:
//   n^2 * vmax^2 < 2^63 (numerator) and n^2 < 2^53 (exact FP64 divisor),
// with vmax = 255 for U8 frames and 1 for BIT1 frames.
bool overflow_ok(int64_t n, int fmt);

struct CorrPlan {
  int64_t n = 0, pa = 0, pb = 0;
  int fmt = 0;
  int64_t pa_pad = 0, pb_pad = 0;   // operand rows
  int64_t kpad_bits = 0;            // frames, padded to kBitBlock
  int64_t kpad_bytes = 0;           // frames, padded to kByteBlock (U8 only)
  int64_t row_bytes_bits = 0;       // kpad_bits / 8
  int64_t row_bytes_bytes = 0;      // kpad_bytes (U8 only)
  int passes = 1;                   // int32 passes for byte operands
  // workspace layout (byte offsets)
  // sums: popcounts of the bit rows; sum2: byte sums (U8 data that is not binary)
  size_t off_sum_a = 0, off_sum_b = 0, off_sum2_a = 0, off_sum2_b = 0, off_stats = 0;
  size_t off_op_a = 0, off_op_b = 0, off_acc64 = 0;
  size_t total = 0;
};

// Fills `p`; returns CPI_OK or an error with `why` set.
cpi_status plan_correlate(int64_t n, int64_t pa, int64_t pb, int fmt, CorrPlan* p,
                          std::string* why);

struct PlainPlan {
  int64_t n = 0, pa = 0, pb = 0;
  int fmt = 0;
  int64_t kpad = 0;                 // frames padded to the FP32 GEMM K tile
  int64_t pa_pad = 0, pb_pad = 0;   // columns padded to the FP32 GEMM tile
  size_t off_fa = 0, off_fb = 0, off_sa = 0, off_sb = 0, total = 0;
};

cpi_status plan_correlate_plain(int64_t n, int64_t pa, int64_t pb, int fmt,
                                PlainPlan* p, std::string* why);

// Refocus: per-plane coordinate tables, and the partial-sum buffer of the
// batched kernel when the view loop is split over work-groups.
struct RefocusPlan {
  int64_t table_stride = 0;         // entries per plane: out_w + out_h + wb + hb
  size_t off_itab = 0, off_ftab = 0, off_ytab = 0, off_bounds = 0, off_partial = 0;
  size_t partial_bytes = 0;         // capacity reserved for partial sums (and the
                                    // row-lane kernel's T of one plane chunk)
  // row-lane kernel: planes per chunk (0: T of 16 planes would exceed 4 GiB),
  // output columns its T rows hold, and its table regions
  int64_t rows_chunk = 0, rows_wout_cap = 0;
  size_t off_rows_xe = 0, off_rows_yr = 0;
  size_t total = 0;
};

constexpr int kMaxViewSplits = 16;

cpi_status validate_geometry(const cpi_geometry* g, std::string* why);
cpi_status validate_alphas(const cpi_geometry* g, const double* alphas, int32_t n_alpha,
                           std::string* why);
cpi_status plan_refocus(const cpi_geometry* g, int32_t n_alpha, RefocusPlan* p,
                        std::string* why);

struct StreamPlan {
  CorrPlan chunk;                   // plan of one chunk of max_chunk frames
  int64_t max_chunk = 0;
  bool state64 = false;             // S_ab state in int64 (U8) or int32 (BIT1)
  size_t off_chunk_ws = 0;          // chunk workspace (operands, chunk sums, stats)
  size_t off_sab = 0, off_sum_a = 0, off_sum_b = 0, off_gamma32 = 0;
  size_t off_stage_a = 0, off_stage_b = 0;   // device copies of host chunks
  size_t off_stage_a2 = 0, off_stage_b2 = 0; // the second pair (copies alternate)
  int gamma_buffers = 1;            // FP32 Gamma buffers (2: pushes alternate; 0: none,
                                    // the pushes fold the sums only)
  size_t off_gamma32b = 0;          // second buffer (== off_gamma32 when one)
  size_t total = 0;
};

cpi_status plan_stream(int64_t pa, int64_t pb, int fmt, int64_t max_chunk,
                       StreamPlan* p, std::string* why, int gamma_buffers = 1);

}  // namespace cpi
