// Device kernels of the CPI library and their host-side launchers.
// Every launcher only enqueues work on `stream` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace cpi {

// ---- fills --------------------------------------------------------------
hipError_t fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s);
hipError_t fill_u64(uint64_t* p, int64_t count, uint64_t v, hipStream_t s);
// Up to kZeroRanges ranges of 64-bit words (8-byte aligned) zeroed in one launch.
constexpr int kZeroRanges = 6;
struct ZeroRanges {
  uint64_t* ptr[kZeroRanges];
  int64_t words[kZeroRanges];
  int count = 0;
  void add(void* p, int64_t n) {
    ptr[count] = static_cast<uint64_t*>(p);
    words[count] = n;
    ++count;
  }
};
hipError_t zero_ranges(const ZeroRanges& z, hipStream_t s);
hipError_t add_i64(int64_t* dst, const int64_t* src, int64_t count, hipStream_t s);

// ---- ingest: frame-major frames -> pixel-major operands ------------------
// One detector's part of an ingest: its frames (n frames of npix pixels,
// frame-major: bytes, or bits packed 8 per byte with each frame padded to
// whole bytes), operand rows (npix_pad rows), bit-row popcount sums and byte
// sums (int64), and whether its bit rows take the FP4 bit exchange (swap02:
// bits 0 and 2 of every 4-bit group of each row word are exchanged, the
// layout of the M operand of the FP4 contraction).  The ingest kernels run
// both detectors' jobs in one launch.
struct IngestJob {
  const uint8_t* frames;
  int64_t npix, npix_pad;
  uint8_t* out;
  int64_t* sums;    // popcounts of the bit rows
  int64_t* sums2;   // byte sums (non-binary data)
  int swap02;
};
// Packed-bit frames -> bit rows (row_bytes = kpad_bits/8), per-pixel popcounts
// added into sums (int64).  Rows [npix, npix_pad) are written too.
hipError_t ingest_bits(const IngestJob& a, const IngestJob& b, int64_t n, int64_t kpad_bits,
                       hipStream_t s);
// Byte frames -> bit rows (bit = low bit of the byte) with per-pixel popcounts
// added into sums, and the OR of every byte accumulated into stats[0].  The
// rows and popcounts are the data exactly when stats[0] <= 1 (binary data);
// stats[0] > 127 exactly when some byte exceeds 127.  swap02 as above.
hipError_t u8_to_bits(const IngestJob& a, const IngestJob& b, int64_t n, int64_t kpad_bits,
                      uint32_t* stats, hipStream_t s);
// Side-by-side sensor frames (frame_h rows of frame_w 1-bit pixels, A the left
// half, B the right) -> BIT1 frames of the roi_w x roi_h region of interest at
// (roi_x, roi_y) inside each half.  Sizes are validated by the caller.
hipError_t split_sidebyside(const uint8_t* frames, int64_t n, int frame_w, int frame_h, int roi_x,
                            int roi_y, int roi_w, int roi_h, uint8_t* out_a, uint8_t* out_b,
                            hipStream_t s);
// Per-pixel byte sums (int64, added into sums2), executed only when
// stats[0] > 1.
hipError_t u8_sums(const IngestJob& a, const IngestJob& b, int64_t n, const uint32_t* stats,
                   hipStream_t s);
// dst[i] = (stats[0] <= 1 ? from_bits : from_bytes)[i]; and dst[i] += the same.
hipError_t select_i64(int64_t* dst, const int64_t* from_bits, const int64_t* from_bytes,
                      int64_t count, const uint32_t* stats, hipStream_t s);
hipError_t add_select_i64(int64_t* dst, const int64_t* from_bits, const int64_t* from_bytes,
                          int64_t count, const uint32_t* stats, hipStream_t s);
// Byte frames -> int8 rows (row_bytes = kpad_bytes), executed only when
// stats[0] > 1; values are offset by -128 when stats[0] > 127; pads are 0.
hipError_t u8_to_bytes(const IngestJob& a, const IngestJob& b, int64_t n, int64_t kpad_bytes,
                       const uint32_t* stats, hipStream_t s);

// ---- int8 MFMA contraction with the exact epilogue -----------------------
enum EpiMode : int {
  EPI_FINAL = 0,        // Gamma from this pass's int32 sums
  EPI_FINAL_ACC64 = 1,  // Gamma from acc64 + this pass
  EPI_STORE64 = 2,      // acc64 = this pass
  EPI_ADD64 = 3,        // acc64 += this pass
  EPI_STREAM32 = 4,     // acc32 += this chunk; gamma_f32 from acc32
  EPI_STREAM64 = 5      // acc64 += un-offset chunk sums; gamma_f32 from acc64
};

struct GemmArgs {
  const uint8_t* opm = nullptr;     // M rows: detector-B pixels (views)
  const uint8_t* opn = nullptr;     // N rows: detector-A pixels
  int64_t row_bytes = 0;
  int64_t k_byte_off = 0;           // first byte of this pass in every row
  int64_t kblocks = 0;              // 64-byte row segments in this pass
  int64_t m_pad = 0, n_pad = 0;     // padded operand rows
  int mode = EPI_FINAL;
  int layout = CPI_GAMMA_VIEW_MAJOR;
  int cond = 0;                     // 0 always; 1 iff stats[0] <= 1; 2 iff stats[0] > 1
  int fp4 = 0;                      // bit rows as FP4 operands (M rows stored with swap02)
  int offset_from_stats = 0;        // byte operands offset by -128 iff stats[0] > 127
  int64_t pa = 0, pb = 0, n = 0;    // n: frames behind the result
  int64_t kchunk = 0;               // frames of this chunk (EPI_STREAM64)
  const int64_t* sum_a = nullptr;   // S_a, S_b of the result (raw, un-offset)
  const int64_t* sum_b = nullptr;
  const int64_t* csum_a = nullptr;  // chunk sums (EPI_STREAM64)
  const int64_t* csum_b = nullptr;
  const uint32_t* stats = nullptr;
  double* gamma = nullptr;
  float* gamma_f32 = nullptr;
  int64_t* numer = nullptr;
  int64_t* acc64 = nullptr;         // view-major Pb x Pa
  int32_t* acc32 = nullptr;         // view-major Pb x Pa
};

// bits: operands are bit rows; otherwise int8 rows.
hipError_t gemm_correlate(const GemmArgs& a, bool bits, hipStream_t s);

// Whether a bit-row contraction over kblocks 512-frame blocks takes the FP4
// encoding (then its M rows must be ingested with swap02) under the current
// matrix-core encoding setting.  Decided once per call by the caller.
bool bits_use_fp4(int64_t kblocks);

// Matrix-core encoding of bit rows (a cpi_mma_encoding value), process-wide.
void set_mma_encoding(int enc);
int get_mma_encoding();

// ---- measured peaks ---------------------------------------------------------
size_t peaks_scratch_bytes(size_t copy_bytes);
// Register-only loops of the int8 and FP4 matrix-core ops, and a device copy
// of copy_bytes; synchronises s.
hipError_t measure_peaks(uint8_t* scratch, size_t copy_bytes, hipStream_t s, double* int8_ops,
                         double* fp4_ops, double* copy_bytes_per_s);

// Gamma from a streaming state (view-major int32 or int64 S_ab, raw sums).
hipError_t state_gamma(const void* sab, bool sab64, const int64_t* sum_a, const int64_t* sum_b,
                       int64_t n, int64_t pa, int64_t pb, int layout, double* gamma,
                       float* gamma_f32, int64_t* numer, hipStream_t s);

// ---- plain FP32 path ------------------------------------------------------
hipError_t unpack_f32(const uint8_t* frames, int fmt, int64_t n, int64_t npix, int64_t kpad,
                      int64_t cols_pad, float* out, float* colsum, hipStream_t s);
hipError_t sgemm_gamma(const float* fb, const float* fa, int64_t kpad, int64_t pb_pad,
                       int64_t pa_pad, int64_t pa, int64_t pb, int64_t n, const float* sa,
                       const float* sb, int layout, float* out, hipStream_t s);

// ---- refocus -------------------------------------------------------------
struct RefGeom {
  int wa, ha, wb, hb, out_w, out_h;
  double mag_x, mag_y, ca_x, ca_y, cb_x, cb_y;
};

// Per-plane coordinate tables for planes [first, first+count), count <= 64:
// integer parts and FP32 fractions of a_x, a_y, b_x, b_y; and, if ytab is
// not null, the row table of the batched kernel (16 bytes per plane, y_b, y_r).
hipError_t refocus_tables(const RefGeom& g, const double* alphas, int first, int count,
                          int64_t stride, int32_t* itab, float* ftab, void* ytab, hipStream_t s);
hipError_t refocus_plain(const float* gamma, const RefGeom& g, const int32_t* itab,
                         const float* ftab, int64_t stride, int plane, float* out,
                         hipStream_t s);

struct RefocusConfig {
  int kp = 4;        // planes per work-group (one wave per plane)
  int rw = 8;        // output rows per work-group tile
  int splits = 1;    // view-row splits (partial sums reduced afterwards)
  int mode = 0;      // 0: per-row interpolation (k_ref_batched); 1: column sums over x_b
                     // first, row weights once per y_b (k_ref_sep); 2: row-lane x pass
                     // and fold (k_ref_rows), with kp planes x rw output columns per
                     // work-group (splits and stages unused)
  int stages = 3;    // mode 1: view windows staged in LDS (2, 3 or 4)
};
bool refocus_config_supported(const RefocusConfig& c);
// bounds: workspace for the window bounds per (plane group, tile column,
// view column) and (plane group, tile row, view row), two ints each; sized
// for plane groups of at least 1 plane and tiles of at least 64 x 8.
hipError_t refocus_batched(const float* gamma, const RefGeom& g, const int32_t* itab,
                           const float* ftab, const void* ytab, void* bounds, int64_t stride,
                           int n_alpha,
                           const RefocusConfig& c, float* partial, float* out,
                           hipStream_t s);

// Row-lane batched refocus (x pass over view rows, then the fold over y_b),
// planes in chunks of `chunk` (a multiple of 16).  Workspace pieces: the
// per-view tables of one chunk (header and pair entries), touched-row ranges,
// and T of one chunk (chunk * hb * ha * wout_cap floats).
struct RowsWorkspace {
  int32_t* xe = nullptr;
  int2* yr = nullptr;
  float* t = nullptr;
  int chunk = 0;
  int64_t wout_cap = 0;
};
bool rows_config_built(int na, int xr);
// Smallest staged window width (16, 32 or 64 columns) that holds every
// column cell of every (group of na planes, xr output columns) at any view,
// or 0 if none does.
int rows_window_width(const RefGeom& g, const double* alphas, int n_alpha, int na, int xr);
// Whether the row-lane kernel with na planes x xr columns per work-group runs
// this geometry and plane set with chunks of `chunk` planes (host check).
bool rows_supported(const RefGeom& g, const double* alphas, int n_alpha, int na, int xr,
                    int64_t chunk);
hipError_t refocus_rows(const float* gamma, const RefGeom& g, const double* alphas,
                        const int32_t* itab, const float* ftab, const void* ytab, int64_t stride,
                        int n_alpha, int na, int xr, const RowsWorkspace& w, float* out,
                        hipStream_t s);

// Gamma views resampled on a lens-plane sample grid (x_b, y_b) = (ox + i sx,
// oy + j sy), i < nx, j < ny: out[j * nx + i][.] = bilinear interpolant of the
// pb = wb * hb views of pa values at that point (zero outside detector B).
hipError_t resample_views(const float* gamma, int64_t pa, int wb, int hb, int nx, int ny, double ox,
                          double oy, double sx, double sy, float* out, hipStream_t s);

// ---- learned denoiser: BF16 matrix-core convolutions and their companions --
// Activations are NHWC bfloat16 (raw uint16 bits); layers keep Cin % 8 == 0
// and Cout % 32 == 0.  Weights fed to the matrix cores are bfloat16 rows of
// length Kpad (a multiple of 32) holding k = tap * Cin + ci, zero beyond
// ks * ks * Cin.
struct NnConvArgs {
  const uint16_t* in = nullptr;    // [B][H][W][Cin]
  const uint16_t* wk = nullptr;    // [Cout][Kpad]
  const float* bias = nullptr;     // [Cout] or null
  const uint16_t* mask = nullptr;  // [B][H][W][Cout]: output zeroed where mask <= 0; or null
  uint16_t* out = nullptr;         // [B][H][W][Cout] bfloat16, or null
  float* out_f32 = nullptr;        // [B][H][W][Cout] FP32, or null
  int B = 0, H = 0, W = 0, Cin = 0, Cout = 0, ks = 0, Kpad = 0;
  int relu = 0;
  // Concatenated input: if low is set, input channels [0, c_low) are the
  // nearest 2x upsampling of low ([B][H/2][W/2][c_low], H and W even) and
  // channels [c_low, Cin) come from in ([B][H][W][Cin - c_low]); c_low % 32
  // == 0.  Only the LDS-staged 3x3 kernels take it (nn_conv_takes_low).
  const uint16_t* low = nullptr;
  int c_low = 0;
  // Pooled input: if set (low unset), in is [B][2H][2W][Cin] and the input
  // is its 2x2 max-pooling.  Also LDS-staged 3x3 kernels only.
  int pool_in = 0;
  // Split output (instead of out, out_f32, bias, ReLU and mask): output
  // channels [0, c1) summed over each 2x2 pixel window (of the values
  // rounded to bfloat16, as ((00 + 01) + (10 + 11))) into dlow
  // [B][H/2][W/2][c1], zeroed where low_mask <= 0 (nullable); channels
  // [c1, Cout) into dskip [B][H][W][Cout - c1].  The gradient of
  // [upsample2(low), skip] in one pass (nn_conv_takes_split).
  uint16_t* dlow = nullptr;
  uint16_t* dskip = nullptr;
  const uint16_t* low_mask = nullptr;
  int c1 = 0;
};
// Forward convolution (zero padding, ks odd); the backward-data
// convolution is the same call on dY with the flipped, transposed weights.
hipError_t nn_conv(const NnConvArgs& a, hipStream_t s);
// whether nn_conv runs this shape on a kernel that reads a concatenated or
// pooled input in place
bool nn_conv_takes_low(const NnConvArgs& a);
// whether nn_conv can write this shape's output split (dlow / dskip)
bool nn_conv_takes_split(const NnConvArgs& a);

struct NnWgradArgs {
  const uint16_t* in = nullptr;    // [B][H][W][Cin] layer input
  const uint16_t* dy = nullptr;    // [B][H][W][Cout] output gradient
  float* dw = nullptr;             // [Cout][ks*ks*Cin], accumulated into
  float* db = nullptr;             // [Cout] bias gradient accumulated into, or null
  // Partial sums of the pixel splits ([split][Cout*ks*ks*Cin + Cout] floats),
  // or null: with it the splits store their tiles and one more kernel adds
  // them to dw and db in split order (deterministic); without it they add
  // with FP32 atomics.
  float* part = nullptr;
  int64_t part_cap = 0;            // floats available at part
  int B = 0, H = 0, W = 0, Cin = 0, Cout = 0, ks = 0, Kpad = 0;
  // concatenated or pooled input as in NnConvArgs (3x3 layers with
  // Cin % 32 == 0 only)
  const uint16_t* low = nullptr;
  int c_low = 0;
  int pool_in = 0;
};
// phases: 1 the splits' kernel, 2 the reduction of the partial buffer into
// dw / db (part set), 3 both (the reduction may go on another stream, after
// the first phase and before the partial buffer is used again)
hipError_t nn_conv_wgrad(const NnWgradArgs& a, hipStream_t s, int phases = 3);
// floats of partial sums nn_conv_wgrad uses for this shape (the part buffer)
int64_t nn_conv_wgrad_part_floats(const NnWgradArgs& a);
// db[n] += sum over the M pixels of dy[m][n]
hipError_t nn_bias_grad(const uint16_t* dy, int64_t M, int C, float* db, hipStream_t s);
// FP32 weights [Cout][ks*ks][Cin] -> bfloat16 [Cout][kpad] and, if wt is not
// null, the flipped transposed [Cin][kpad_t] (k = tap' * Cout + co with
// tap' = ks*ks - 1 - tap) of the backward-data convolution.
hipError_t nn_pack_weights(const float* w, int Cout, int Cin, int ks, uint16_t* wf, int kpad,
                           uint16_t* wt, int kpad_t, hipStream_t s);
hipError_t nn_maxpool(const uint16_t* in, int B, int H, int W, int C, uint16_t* out,
                      hipStream_t s);
hipError_t nn_maxpool_bwd(const uint16_t* in, int B, int H, int W, int C, const uint16_t* dout,
                          uint16_t* din, hipStream_t s);
// H, W: the input size of the upsampling (output 2H x 2W)
hipError_t nn_upsample(const uint16_t* in, int B, int H, int W, int C, uint16_t* out,
                       hipStream_t s);
hipError_t nn_upsample_bwd(const uint16_t* dout, int B, int H, int W, int C, const uint16_t* mask,
                           uint16_t* din, hipStream_t s);
hipError_t nn_concat(const uint16_t* a, const uint16_t* b, int64_t P, int C1, int C2, uint16_t* out,
                     hipStream_t s);
hipError_t nn_split(const uint16_t* d, int64_t P, int C1, int C2, uint16_t* da, uint16_t* db,
                    hipStream_t s);
// Nearest 2x upsampling of low [B][H][W][C1] concatenated with skip
// [B][2H][2W][C2] into out [B][2H][2W][C1+C2], and its gradient (dlow masked
// by mask <= 0 if given); C1, C2 multiples of 8.
hipError_t nn_upcat(const uint16_t* low, const uint16_t* skip, int B, int H, int W, int C1, int C2,
                    uint16_t* out, hipStream_t s);
hipError_t nn_upcat_grad(const uint16_t* d, int B, int H, int W, int C1, int C2,
                         const uint16_t* mask, uint16_t* dlow, uint16_t* dskip, hipStream_t s);
// the first 3x3 layer: one input channel used (stride cx), 32 outputs, ReLU
hipError_t nn_in1_fwd(const uint16_t* x, int B, int H, int W, int cx, const uint16_t* wk, int kpad,
                      const float* bias, uint16_t* out, hipStream_t s);
// work-groups (partial rows of 32 * 9 * cx + 32 floats) nn_in1_wgrad uses
int nn_in1_wgrad_groups(int64_t P);
// its weight (dw [32][9 * cx]) and bias (db [32]) gradients added in, via part
hipError_t nn_in1_wgrad(const uint16_t* x, int B, int H, int W, int cx, const uint16_t* dy,
                        float* part, float* dw, float* db, hipStream_t s, int phases = 3);
// din = (dout routed to each 2x2 window's first maximal position) + skip,
// zeroed where in <= 0; C % 8 == 0
hipError_t nn_pool_bwd_add(const uint16_t* in, int B, int H, int W, int C, const uint16_t* dout,
                           const uint16_t* skip, uint16_t* din, hipStream_t s);
// the output layer (1x1 to one channel of 32): y[p] = bias[0] + sum_c w[c] h[p][c]
hipError_t nn_out1_fwd(const uint16_t* h, const uint16_t* w, const float* bias, int64_t P, float* y,
                       hipStream_t s);
// work-groups (rows of 36 partial-sum floats) nn_out1_bwd uses for P pixels
int nn_out1_bwd_groups(int64_t P);
// loss (added to *loss), output-layer input gradient gin [P][32] and its
// weight (dw[0 .. 31]) and bias (db[0]) gradients added in, via part
hipError_t nn_out1_bwd(const float* y, const float* res, const float* t, int64_t P,
                       const uint16_t* h, const uint16_t* w, uint16_t* gin, float* loss,
                       float* part, float* dw, float* db, hipStream_t s);
hipError_t nn_add_mask(uint16_t* x, const uint16_t* add, const uint16_t* mask, int64_t n,
                       hipStream_t s);
hipError_t nn_mse(const float* y, int C, const float* res, const float* t, int64_t P, float* loss,
                  uint16_t* dy, hipStream_t s);
hipError_t nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                   float b2, float eps, float c1, float c2, hipStream_t s);
// scratch: nn_normalize_scratch_bytes(B) bytes of device memory (partial sums)
size_t nn_normalize_scratch_bytes(int B);
hipError_t nn_normalize(const float* planes, int B, int64_t hw, int C, uint16_t* out, float* xf,
                        const float* targets, float* tnorm, float* stats, double* scratch,
                        hipStream_t s);
// Weight packing of every layer of a network in one launch: layer l's
// forward rows go to packed + wf_off and, if transposed, its backward-data
// rows to packed + wt_off; its elements are [begin, begin + cout * kpad
// (+ cin * kpad_t)) of the launch's index range.
struct NnPackLayer {
  int64_t w_off = 0, wf_off = 0, wt_off = 0, begin = 0;
  int cout = 0, cin = 0, ks = 0, kpad = 0, kpad_t = 0, transposed = 0;
};
struct NnPackTable {
  NnPackLayer layer[16];
  int n = 0;
  int64_t total = 0;
};
hipError_t nn_pack_all(const float* params, uint16_t* packed, const NnPackTable& tab,
                       hipStream_t s);
hipError_t nn_denormalize(const float* x, int C, const float* res, const float* stats, int64_t hw,
                          int B, float* y, hipStream_t s);
hipError_t nn_quality(const float* pred, const float* target, int B, int H, int W, double* psnr,
                      double* ssim, hipStream_t s);

}  // namespace cpi
