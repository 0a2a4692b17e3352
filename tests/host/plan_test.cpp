// Host-only checks of the planning and validation layer (no HIP): overflow
// bounds, padding, workspace layouts (ordered, 256-byte aligned, large enough
// for every region) and the validation errors.  Built with the sanitizers.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "plan.h"

static int failures = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                 \
    }                                                             \
  } while (0)

using namespace cpi;

static bool aligned(size_t x) { return (x & 255) == 0; }

int main() {
  std::string why;
  // overflow bounds: u8 n^2 * 255^2 < 2^63, both formats n^2 < 2^53
  CHECK(overflow_ok(11909805, CPI_FRAMES_U8));
  CHECK(!overflow_ok(11909806, CPI_FRAMES_U8));
  CHECK(overflow_ok(94906265, CPI_FRAMES_BIT1));
  CHECK(!overflow_ok(94906266, CPI_FRAMES_BIT1));
  CHECK(!overflow_ok(0, CPI_FRAMES_BIT1));

  // correlation plans
  for (int fmt : {0, 1}) {
    for (int64_t n : {1L, 63L, 64L, 511L, 512L, 20000L, 131008L, 131009L, 300000L}) {
      for (int64_t pa : {1L, 255L, 256L, 16384L}) {
        const int64_t pb = 77;
        if (fmt == 0 && !overflow_ok(n, fmt)) continue;
        CorrPlan p;
        CHECK(plan_correlate(n, pa, pb, fmt, &p, &why) == CPI_OK);
        CHECK(p.pa_pad % kRowPad == 0 && p.pa_pad >= pa && p.pa_pad - pa < kRowPad);
        CHECK(p.pb_pad % kRowPad == 0 && p.pb_pad >= pb);
        CHECK(p.kpad_bits % kBitBlock == 0 && p.kpad_bits >= n && p.kpad_bits - n < kBitBlock);
        CHECK(p.row_bytes_bits * 8 == p.kpad_bits);
        const size_t offs[] = {p.off_sum_a, p.off_sum_b, p.off_sum2_a, p.off_sum2_b,
                               p.off_stats, p.off_op_a, p.off_op_b, p.off_acc64, p.total};
        for (size_t i = 0; i + 1 < sizeof(offs) / sizeof(offs[0]); ++i) {
          CHECK(aligned(offs[i]));
          CHECK(offs[i] <= offs[i + 1]);
        }
        int64_t row = p.row_bytes_bits;
        if (fmt == CPI_FRAMES_U8) {
          CHECK(p.kpad_bytes % kByteBlock == 0 && p.kpad_bytes >= n);
          CHECK(p.passes == int((n + kByteChunk - 1) / kByteChunk));
          if (p.row_bytes_bytes > row) row = p.row_bytes_bytes;
          CHECK(p.off_sum2_b - p.off_sum2_a >= size_t(p.pa_pad) * 8);
          if (p.passes > 1) CHECK(p.total - p.off_acc64 >= size_t(pa * pb * 8));
        }
        CHECK(p.off_op_b - p.off_op_a >= size_t(p.pa_pad * row));
        CHECK(p.off_acc64 - p.off_op_b >= size_t(p.pb_pad * row));
        CHECK(p.off_sum_b - p.off_sum_a >= size_t(p.pa_pad) * 8);
      }
    }
  }
  // the byte-chunk bound keeps int32 partial sums below 2^31 for offset bytes
  CHECK(double(kByteChunk) * 128.0 * 128.0 < 2147483647.0);
  CHECK(kByteChunk % kByteBlock == 0);

  CorrPlan p;
  CHECK(plan_correlate(0, 1, 1, 0, &p, &why) == CPI_ERR_INVALID_ARG);
  CHECK(plan_correlate(1, 0, 1, 0, &p, &why) == CPI_ERR_INVALID_ARG);
  CHECK(plan_correlate(1, 1, 1, 9, &p, &why) == CPI_ERR_INVALID_ARG);
  CHECK(plan_correlate(12000000, 1, 1, 0, &p, &why) == CPI_ERR_OVERFLOW);
  CHECK(plan_correlate(1, int64_t(1) << 29, 1, 0, &p, &why) == CPI_ERR_INVALID_ARG);
  CHECK(plan_correlate(1, 1, 1, 0, nullptr, &why) == CPI_ERR_INVALID_ARG);

  PlainPlan pp;
  CHECK(plan_correlate_plain(20000, 16384, 4096, 0, &pp, &why) == CPI_OK);
  CHECK(pp.kpad % 16 == 0 && pp.pa_pad % 128 == 0 && pp.pb_pad % 128 == 0);
  CHECK(pp.off_fb - pp.off_fa >= size_t(pp.kpad * pp.pa_pad * 4));
  CHECK(aligned(pp.off_fb) && aligned(pp.off_sa) && aligned(pp.off_sb));

  // refocus plans and validation
  cpi_geometry g{128, 128, 64, 64, 2.0, 2.0, 63.5, 63.5, 31.5, 31.5, 128, 128};
  RefocusPlan rp;
  CHECK(plan_refocus(&g, 32, &rp, &why) == CPI_OK);
  CHECK(rp.table_stride == 128 + 128 + 64 + 64);
  CHECK(rp.off_ftab - rp.off_itab >= size_t(32 * rp.table_stride * 4));
  CHECK(rp.off_bounds - rp.off_ytab >= size_t(32) * 64 * 128 * 16);
  CHECK(rp.total - rp.off_partial >= rp.partial_bytes);
  // the split partial sums (16 x 32 planes x 128 x 128 floats) or the
  // row-lane kernel's T of one chunk (32 planes x hb 64 x ha 128 x 128
  // output columns), whichever is larger
  CHECK(rp.rows_chunk == 32 && rp.rows_wout_cap == 128);
  CHECK(rp.partial_bytes == std::max(size_t(16) * 32 * 128 * 128 * 4,
                                     size_t(32) * 64 * 128 * 128 * 4));
  CHECK(rp.off_rows_xe >= rp.off_partial + rp.partial_bytes);
  CHECK(rp.off_rows_yr - rp.off_rows_xe >= size_t(32) * 128 * 64 * 12 + size_t(32) * 128 * 64 / 64 * 16);
  CHECK(rp.total - rp.off_rows_yr >= size_t(32) * 64 * 8);
  CHECK(aligned(rp.off_rows_xe) && aligned(rp.off_rows_yr));
  // 128 planes at 256 x 256 on both detectors: T of 64 planes (4 GiB)
  cpi_geometry gp{256, 256, 256, 256, 1.0, 1.0, 127.5, 127.5, 127.5, 127.5, 256, 256};
  CHECK(plan_refocus(&gp, 128, &rp, &why) == CPI_OK);
  CHECK(rp.rows_chunk == 64 && rp.partial_bytes == size_t(64) * 256 * 256 * 256 * 4);
  // 300 planes of a small geometry: chunks of at most 256 planes
  CHECK(plan_refocus(&g, 300, &rp, &why) == CPI_OK);
  CHECK(rp.rows_chunk == 256);
  // views too tall for T of 16 planes within 4 GiB: no row-lane chunks
  cpi_geometry gt{512, 4096, 128, 128, 4.0, 32.0, 255.5, 2047.5, 63.5, 63.5, 512, 4096};
  CHECK(plan_refocus(&gt, 8, &rp, &why) == CPI_OK);
  CHECK(rp.rows_chunk == 0);
  CHECK(plan_refocus(&g, 0, &rp, &why) == CPI_ERR_INVALID_ARG);
  CHECK(plan_refocus(&g, 4097, &rp, &why) == CPI_ERR_INVALID_ARG);
  cpi_geometry bad = g;
  bad.mag_x = NAN;
  CHECK(validate_geometry(&bad, &why) == CPI_ERR_INVALID_ARG);
  bad = g;
  bad.out_w = 0;
  CHECK(validate_geometry(&bad, &why) == CPI_ERR_INVALID_ARG);
  double al[3] = {0.5, 1.0, 1.5};
  CHECK(validate_alphas(&g, al, 3, &why) == CPI_OK);
  al[1] = INFINITY;
  CHECK(validate_alphas(&g, al, 3, &why) == CPI_ERR_INVALID_ARG);
  al[1] = 1e9;
  CHECK(validate_alphas(&g, al, 3, &why) == CPI_ERR_INVALID_ARG);

  // stream plans
  StreamPlan sp;
  CHECK(plan_stream(16384, 4096, 1, 1000, &sp, &why) == CPI_OK);
  CHECK(!sp.state64);
  CHECK(sp.off_sum_a - sp.off_sab >= size_t(16384) * 4096 * 4);
  CHECK(sp.off_stage_a - sp.off_gamma32 >= size_t(16384) * 4096 * 4);
  CHECK(sp.total - sp.off_stage_b >= size_t(1000) * 512);
  CHECK(plan_stream(64, 16, 0, 200000, &sp, &why) == CPI_ERR_INVALID_ARG);
  CHECK(plan_stream(64, 16, 0, 1000, &sp, &why) == CPI_OK && sp.state64);
  CHECK(plan_stream(64, 16, 1, 0, &sp, &why) == CPI_ERR_INVALID_ARG);
  // two FP32 Gamma buffers: the second one past the staging copies
  StreamPlan sp1, sp2;
  CHECK(plan_stream(16384, 4096, 1, 1000, &sp1, &why) == CPI_OK);
  CHECK(sp1.gamma_buffers == 1 && sp1.off_gamma32b == sp1.off_gamma32);
  CHECK(plan_stream(16384, 4096, 1, 1000, &sp2, &why, 2) == CPI_OK);
  CHECK(sp2.gamma_buffers == 2 && sp2.off_gamma32 == sp1.off_gamma32);
  CHECK(sp2.off_gamma32b >= sp2.off_stage_b + size_t(1000) * 512);
  CHECK(sp2.total - sp2.off_gamma32b >= size_t(16384) * 4096 * 4);
  CHECK(sp2.total - sp1.total >= size_t(16384) * 4096 * 4);
  CHECK(plan_stream(64, 16, 1, 100, &sp, &why, 3) == CPI_ERR_INVALID_ARG);
  CHECK(plan_stream(64, 16, 1, 100, &sp, &why, -1) == CPI_ERR_INVALID_ARG);
  // no FP32 Gamma buffer (blocked correlation): the state is S_ab, the sums
  // and one block's operands
  StreamPlan sp0;
  CHECK(plan_stream(16384, 4096, 1, 1000, &sp0, &why, 0) == CPI_OK);
  CHECK(sp0.gamma_buffers == 0 && sp1.total - sp0.total >= size_t(16384) * 4096 * 4);
  CHECK(sp0.total - sp0.off_sab >= size_t(16384) * 4096 * 4);

  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("plan tests passed\n");
  return 0;
}
