// Row-lane batched refocus: the shift-and-sum of the perspective views of
// Gamma (the refocusing of the paper's Section 4.1) in two passes.
//
// The interpolation weights of a sample factor into a column side that
// depends on (plane, x_r, x_b) and a row side that depends on
// (plane, y_r, y_b), and the tap positions likewise.  So
//     T(plane, y_b, y, x_r) = sum over x_b of  wx0 * view(y, xc) + wx1 * view(y, xc + 1)
// (view = Gamma(., x_b, y_b), xc, wx0, wx1 the clamped column cell of
// (plane, x_r, x_b)) is computed for every view row y first, and then
//     out(plane, y_r, x_r) = sum over y_b of  wy0 * T(.., yc, x_r) + wy1 * T(.., yc + 1, x_r)
// with (yc, wy0, wy1) the clamped row cell of (plane, y_r, y_b).
//
// x pass (k_ref_rows).  A work-group owns one lens-plane row y_b, a band of
// 128 view rows, a group of NA planes and XR consecutive output columns:
// P = NA * XR (plane, column) pairs, 64 per wave.  Each lane holds two view
// rows, so for a given view and pair the column cell is the same for every
// lane.  Cells and weights come from a per-view table (k_rows_xtab) staged
// in LDS beside the window: three 16-byte reads per lane and view put 16
// pairs' values in each register, one pair per lane of a row of 16, and a
// DPP row broadcast hands a pair's value to every lane as an operand of the
// address add and of the multiply-adds, so the table costs no LDS traffic
// per tap.  For every view x_b the work-group stages a window of the band's
// rows and WW columns (the union of its pairs' cells) in LDS, two stages
// deep, stored column by column: two single 8-byte reads give a lane both
// taps of both its rows.  The window is loaded with coalesced 16-byte reads
// (16 rows x 64 bytes per instruction) into registers while the previous
// view is interpolated, and stored transposed; a column stride of 132 floats
// keeps those stores free of bank conflicts.  Work-groups are mapped so that
// all those of one y_b run on one XCD and share its L2.
//
// Fold pass (k_ref_rows_fold): one thread per output pixel of a plane sums
// the two T rows of each y_b with the row weights.
//
// Planes are processed in chunks whose T fits the caller's workspace.  Both
// sums run in a fixed order (x_b, then y_b), so results are bitwise
// reproducible for a given configuration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <utility>

#include "kernels.h"
#include "refocus_common.h"

namespace cpi {

namespace {

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kRowsBand = 128;       // view rows per work-group (two per lane)
constexpr int kBufferWord3 = 0x00020000;   // buffer descriptor word 3 for gfx9 (32-bit data)
constexpr int kRowsColStride = 132;  // LDS floats per window column (even; 132 = 4 mod 64)

// (plane, column) pairs per wave: 64 for work-groups of 256 pairs, else 32,
// so that a work-group of 128 pairs has four waves and two such work-groups
// (their LDS fits a CU twice) keep two waves on every SIMD.
constexpr int rows_pairs_per_wave(int pairs) { return pairs >= 256 ? 64 : 32; }

// Column cells of every (plane, output column) pair of work-group (group gq,
// tile t) against lens-plane column x_b: a 4-word header (window start, and
// one bit per 8-pair chunk with a nonzero weight), then per pair the byte offset of its cell's column in the window
// and its two weights (zero for pairs
// past the planes or columns, or whose taps fall outside the view).  One
// block per (gq, t, x_b), one thread per pair.  The arithmetic is that of the
// other refocus kernels.
template <int NA, int XR>
__global__ __launch_bounds__(NA * XR) void k_rows_xtab(GeomI g, const int32_t* __restrict__ itab,
                                                     const float* __restrict__ ftab,
                                                     int64_t stride, int first, int count,
                                                     int tiles, int ww,
                                                     int32_t* __restrict__ xe) {
  constexpr int P = NA * XR;
  const int64_t idx = blockIdx.x;
  const int xb = int(idx % g.wb);
  const int t = int((idx / g.wb) % tiles);
  const int gq = int(idx / (int64_t(g.wb) * tiles));
  const int p = threadIdx.x;
  const int k = p / XR, j = p % XR;
  const int pl = gq * NA + k;
  const int xr = t * XR + j;
  int c = 0;
  float w0 = 0.0f, w1 = 0.0f;
  if (pl < count && xr < g.out_w) {
    const int32_t* it = itab + int64_t(first + pl) * stride;
    const float* ft = ftab + int64_t(first + pl) * stride;
    const int e_bx = g.out_w + g.out_h;
    int x0 = it[xr] + it[e_bx + xb];
    float fx = ft[xr] + ft[e_bx + xb];
    if (fx >= 1.0f) {
      x0 += 1;
      fx -= 1.0f;
    }
    clamp_cell(x0, fx, g.wa, c, w0, w1);
  }
  const bool live = w0 != 0.0f || w1 != 0.0f;
  __shared__ int smin, smax;
  __shared__ unsigned slive;
  if (p == 0) {
    smin = 1 << 30;
    smax = -(1 << 30);
    slive = 0u;
  }
  __syncthreads();
  if (live) {
    atomicMin(&smin, c);
    atomicMax(&smax, c);
    atomicOr(&slive, 1u << (p / 8));
  }
  __syncthreads();
  int wx0 = slive ? smin : 0;
  if (wx0 > g.wa - ww) wx0 = g.wa - ww;
  if (wx0 < 0) wx0 = 0;
  // The host's window bound keeps every cell in the window; the clamp keeps
  // LDS reads inside it regardless.
  int rel = live ? c - wx0 : 0;
  rel = rel < 0 ? 0 : (rel > ww - 2 ? ww - 2 : rel);
  // per wave slice of PW pairs: offsets, w0, w1, each PW words with pair
  // 16 k + i of the slice at word NK i + k (NK = PW / 16: one read of NK
  // words per lane gives lane i of every row of 16 the pairs it broadcasts)
  constexpr int PW = rows_pairs_per_wave(P), NK = PW / 16;
  int32_t* e = xe + idx * (4 + 3 * P);
  const int q = p % PW, slot = 4 + 3 * PW * (p / PW) + NK * (q % 16) + q / 16;
  e[slot] = rel * kRowsColStride * 4;
  e[slot + PW] = __builtin_bit_cast(int32_t, live ? w0 : 0.0f);
  e[slot + 2 * PW] = __builtin_bit_cast(int32_t, live ? w1 : 0.0f);
  if (p == 0) {
    e[0] = wx0;
    e[1] = int32_t(slive);
    e[2] = 0;
    e[3] = 0;
  }
}

// View rows [lo, hi] that any output row of the group's planes samples with
// a nonzero weight at lens-plane row y_b (lo > hi if none).  One block per
// (gq, y_b).
__global__ __launch_bounds__(256) void k_rows_yrange(GeomI g, const YEntry* __restrict__ ytab,
                                                     int first, int count, int na,
                                                     int2* __restrict__ yr) {
  const int gq = int(blockIdx.x / g.hb), yb = int(blockIdx.x % g.hb);
  int lo = 1 << 30, hi = -(1 << 30);
  for (int e = threadIdx.x; e < na * g.out_h; e += blockDim.x) {
    const int k = e / g.out_h, y = e % g.out_h;
    const int pl = gq * na + k;
    if (pl >= count) continue;
    const YEntry v = ytab[(int64_t(first + pl) * g.hb + yb) * g.out_h + y];
    if (v.w0 != 0.0f) {
      lo = min(lo, v.row);
      hi = max(hi, v.row);
    }
    if (v.w1 != 0.0f) {
      lo = min(lo, v.row + 1);
      hi = max(hi, v.row + 1);
    }
  }
  __shared__ int slo, shi;
  if (threadIdx.x == 0) {
    slo = 1 << 30;
    shi = -(1 << 30);
  }
  __syncthreads();
  atomicMin(&slo, lo);
  atomicMax(&shi, hi);
  __syncthreads();
  if (threadIdx.x == 0) yr[blockIdx.x] = make_int2(slo, shi);
}

template <int NA, int XR, int WW>
struct RowsShape {
  static constexpr int P = NA * XR;               // (plane, column) pairs
  static constexpr int PW = rows_pairs_per_wave(P);   // pairs per wave
  static constexpr int NK = PW / 16;              // table values per lane and kind
  static constexpr int NSTEP = PW / 4;            // steps (4 pairs each) per view
  static constexpr int NPS = P / PW;              // waves
  static constexpr int TAB = 4 + 3 * P;           // table words per view (header, offsets, w0, w1)
  static constexpr int WIN = WW * kRowsColStride;    // window floats per stage
  static constexpr int STAGE = WIN + TAB;         // floats per stage
  static constexpr int NCP = 2 * (WW / 4);        // 16-row x 64-byte copies per view
  static constexpr int CPW = NCP / NPS;           // copies per wave per view
  static constexpr int PH = CPW > 8 ? CPW / 8 : 1;  // copy phases per view (8 copies each)
  static constexpr int CPH = CPW / PH;            // copies per phase
  static constexpr int NM = 8 / NPS;              // row blocks a wave copies
  static_assert(P % 64 == 0 && P <= 256 && (XR % 64 == 0 || 64 % XR == 0) && XR % 4 == 0,
                "pair layout");
  static_assert(WW == 16 || WW == 32 || WW == 64, "window width");
  static_assert(NPS <= 8 && NCP % NPS == 0 && CPW % PH == 0 && NSTEP % PH == 0,
                "copies per wave");
  static_assert(TAB / 4 <= NPS * 64, "table copy");
  static_assert(2 * STAGE * 4 <= 160 * 1024, "LDS");
};

typedef int i4 __attribute__((ext_vector_type(4)));
template <int N>
using ivec = int __attribute__((ext_vector_type(N)));
template <int N>
using fvec = float __attribute__((ext_vector_type(N)));

// The per-view table of a wave's PW pairs, as read by each lane: component k
// of lane 16 r + i belongs to pair 16 k + i (every row of 16 lanes holds the
// same values).  A DPP row broadcast (lane i of each row to the whole row)
// then makes a pair's value an operand of every lane's instruction: the
// column offset of its cell for the tap address, its weights for the
// multiply-adds.
template <int NK>
struct RowsTab {
  ivec<NK> off;     // byte offset of the cell's column in the window
  fvec<NK> w0, w1;  // weights of the cell's two columns
};
struct RowsTaps {
  f2 lo[4], hi[4];   // rows 2 lane, 2 lane + 1 at the cell's column / the next
};

#define CPI_ROWS_READS                           \
  "ds_read_b64 %[t0], %[a0]\n"                   \
  "ds_read_b64 %[u0], %[a0] offset:528\n"        \
  "ds_read_b64 %[t1], %[a1]\n"                   \
  "ds_read_b64 %[u1], %[a1] offset:528\n"        \
  "ds_read_b64 %[t2], %[a2]\n"                   \
  "ds_read_b64 %[u2], %[a2] offset:528\n"        \
  "ds_read_b64 %[t3], %[a3]\n"                   \
  "ds_read_b64 %[u3], %[a3] offset:528\n"
#define CPI_ROWS_ADDRS                                                            \
  "v_add_u32_dpp %[b0], %[of], %[lb] row_newbcast:%[m0] row_mask:0xf bank_mask:0xf\n" \
  "v_add_u32_dpp %[b1], %[of], %[lb] row_newbcast:%[m1] row_mask:0xf bank_mask:0xf\n" \
  "v_add_u32_dpp %[b2], %[of], %[lb] row_newbcast:%[m2] row_mask:0xf bank_mask:0xf\n" \
  "v_add_u32_dpp %[b3], %[of], %[lb] row_newbcast:%[m3] row_mask:0xf bank_mask:0xf\n"
#define CPI_ROWS_FMA(c, w, v, n) \
  "v_fmac_f32_dpp %[" c "], %[" w "], %[" v "] row_newbcast:%[" n "] row_mask:0xf bank_mask:0xf\n"
#define CPI_ROWS_FMAS                                                            \
  CPI_ROWS_FMA("c00", "x", "l0x", "n0") CPI_ROWS_FMA("c10", "x", "l0y", "n0")   \
  CPI_ROWS_FMA("c00", "y", "h0x", "n0") CPI_ROWS_FMA("c10", "y", "h0y", "n0")   \
  CPI_ROWS_FMA("c01", "x", "l1x", "n1") CPI_ROWS_FMA("c11", "x", "l1y", "n1")   \
  CPI_ROWS_FMA("c01", "y", "h1x", "n1") CPI_ROWS_FMA("c11", "y", "h1y", "n1")   \
  CPI_ROWS_FMA("c02", "x", "l2x", "n2") CPI_ROWS_FMA("c12", "x", "l2y", "n2")   \
  CPI_ROWS_FMA("c02", "y", "h2x", "n2") CPI_ROWS_FMA("c12", "y", "h2y", "n2")   \
  CPI_ROWS_FMA("c03", "x", "l3x", "n3") CPI_ROWS_FMA("c13", "x", "l3y", "n3")   \
  CPI_ROWS_FMA("c03", "y", "h3x", "n3") CPI_ROWS_FMA("c13", "y", "h3y", "n3")
#define CPI_ROWS_ACC_OUT                                                                   \
  [c00] "+v"(acc0[p]), [c01] "+v"(acc0[p + 1]), [c02] "+v"(acc0[p + 2]),                   \
      [c03] "+v"(acc0[p + 3]), [c10] "+v"(acc1[p]), [c11] "+v"(acc1[p + 1]),               \
      [c12] "+v"(acc1[p + 2]), [c13] "+v"(acc1[p + 3])
#define CPI_ROWS_FMA_IN                                                                    \
  [x] "v"(tb.w0[K]), [y] "v"(tb.w1[K]), [n0] "i"(I), [n1] "i"(I + 1), [n2] "i"(I + 2),     \
      [n3] "i"(I + 3), [l0x] "v"(cur.lo[0].x), [l0y] "v"(cur.lo[0].y),                     \
      [l1x] "v"(cur.lo[1].x), [l1y] "v"(cur.lo[1].y), [l2x] "v"(cur.lo[2].x),              \
      [l2y] "v"(cur.lo[2].y), [l3x] "v"(cur.lo[3].x), [l3y] "v"(cur.lo[3].y),              \
      [h0x] "v"(cur.hi[0].x), [h0y] "v"(cur.hi[0].y), [h1x] "v"(cur.hi[1].x),              \
      [h1y] "v"(cur.hi[1].y), [h2x] "v"(cur.hi[2].x), [h2y] "v"(cur.hi[2].y),              \
      [h3x] "v"(cur.hi[3].x), [h3y] "v"(cur.hi[3].y)
#define CPI_ROWS_READ_OUT                                                                  \
  [t0] "=&v"(nx.lo[0]), [t1] "=&v"(nx.lo[1]), [t2] "=&v"(nx.lo[2]), [t3] "=&v"(nx.lo[3]), \
      [u0] "=&v"(nx.hi[0]), [u1] "=&v"(nx.hi[1]), [u2] "=&v"(nx.hi[2]), [u3] "=&v"(nx.hi[3])

// A wave's pass over its PW pairs for one view, 4 pairs (chunk C) per step.
// Each step is one inline-asm block that issues the 8 tap reads of chunk
// C + 1 (both rows of a lane at the cell's column and at the next: single
// 8-byte reads, which run at twice the rate of the paired form the compiler
// would merge them into), forms the tap addresses of chunk C + 2, does the 16
// multiply-adds of chunk C on values read by the previous step, then waits
// for its reads: the LDS latency of one chunk overlaps the arithmetic of the
// previous one.  (DPP operands here are only ever written by LDS reads, or
// by VALU instructions at least two instructions earlier.)
template <int C, int NSTEP, int NK, int PW>
__device__ __forceinline__ void rows_step(uint32_t lbase, const RowsTab<NK>& tb, RowsTaps& cur,
                                          uint32_t (&addr)[4], float (&acc0)[PW],
                                          float (&acc1)[PW]) {
  constexpr int p = 4 * C;
  constexpr int K = C / 4, I = 4 * (C % 4);             // chunk C's pairs: component, lanes
  constexpr int K2 = (C + 2) / 4, I2 = 4 * ((C + 2) % 4); // chunk C + 2's
  if constexpr (C == NSTEP - 1) {
    asm volatile("s_nop 1\n" CPI_ROWS_FMAS : CPI_ROWS_ACC_OUT : CPI_ROWS_FMA_IN);
  } else if constexpr (C == NSTEP - 2) {
    RowsTaps nx;
    asm volatile(CPI_ROWS_READS CPI_ROWS_FMAS "s_waitcnt lgkmcnt(0)"
                 : CPI_ROWS_READ_OUT, CPI_ROWS_ACC_OUT
                 : [a0] "v"(addr[0]), [a1] "v"(addr[1]), [a2] "v"(addr[2]), [a3] "v"(addr[3]),
                   CPI_ROWS_FMA_IN);
    cur = nx;
  } else {
    RowsTaps nx;
    uint32_t na[4];
    asm volatile(CPI_ROWS_READS CPI_ROWS_ADDRS CPI_ROWS_FMAS "s_waitcnt lgkmcnt(0)"
                 : CPI_ROWS_READ_OUT, [b0] "=&v"(na[0]), [b1] "=&v"(na[1]), [b2] "=&v"(na[2]),
                   [b3] "=&v"(na[3]), CPI_ROWS_ACC_OUT
                 : [a0] "v"(addr[0]), [a1] "v"(addr[1]), [a2] "v"(addr[2]), [a3] "v"(addr[3]),
                   [of] "v"(tb.off[K2]), [lb] "v"(lbase), [m0] "i"(I2), [m1] "i"(I2 + 1),
                   [m2] "i"(I2 + 2), [m3] "i"(I2 + 3), CPI_ROWS_FMA_IN);
    cur = nx;
#pragma unroll
    for (int j = 0; j < 4; ++j) addr[j] = na[j];
  }
}

// tbl: this lane's slot (NK words) of the wave's table slice; lbase: this
// lane's two rows in the window's first column.  after(integral_constant<C>)
// runs after step C (the next view's copies are spread over the pass).
template <int NK, int PW, typename After, int... C>
__device__ __forceinline__ void rows_view(uint32_t tbl, uint32_t lbase, float (&acc0)[PW],
                                          float (&acc1)[PW], After&& after,
                                          std::integer_sequence<int, C...>) {
  constexpr int NSTEP = sizeof...(C);
  static_assert(NSTEP == PW / 4 && NK == PW / 16, "pass shape");
  RowsTab<NK> tb;
  if constexpr (NK == 4) {
    asm volatile("ds_read_b128 %0, %3\n"
                 "ds_read_b128 %1, %3 offset:256\n"
                 "ds_read_b128 %2, %3 offset:512\n"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(tb.off), "=&v"(tb.w0), "=&v"(tb.w1)
                 : "v"(tbl));
  } else {
    asm volatile("ds_read_b64 %0, %3\n"
                 "ds_read_b64 %1, %3 offset:128\n"
                 "ds_read_b64 %2, %3 offset:256\n"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(tb.off), "=&v"(tb.w0), "=&v"(tb.w1)
                 : "v"(tbl));
  }
  // tap addresses of chunks 0 and 1, then chunk 0's taps
  uint32_t a[4], addr[4];
  asm volatile(
      "s_nop 1\n"
      "v_add_u32_dpp %[a0], %[of], %[lb] row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
      "v_add_u32_dpp %[a1], %[of], %[lb] row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
      "v_add_u32_dpp %[a2], %[of], %[lb] row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
      "v_add_u32_dpp %[a3], %[of], %[lb] row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
      "v_add_u32_dpp %[b0], %[of], %[lb] row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
      "v_add_u32_dpp %[b1], %[of], %[lb] row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
      "v_add_u32_dpp %[b2], %[of], %[lb] row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
      "v_add_u32_dpp %[b3], %[of], %[lb] row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
      : [a0] "=&v"(a[0]), [a1] "=&v"(a[1]), [a2] "=&v"(a[2]), [a3] "=&v"(a[3]),
        [b0] "=&v"(addr[0]), [b1] "=&v"(addr[1]), [b2] "=&v"(addr[2]), [b3] "=&v"(addr[3])
      : [of] "v"(tb.off[0]), [lb] "v"(lbase));
  RowsTaps cur;
  asm volatile(
      "s_nop 1\n"
      "ds_read_b64 %[t0], %[a0]\n"
      "ds_read_b64 %[u0], %[a0] offset:528\n"
      "ds_read_b64 %[t1], %[a1]\n"
      "ds_read_b64 %[u1], %[a1] offset:528\n"
      "ds_read_b64 %[t2], %[a2]\n"
      "ds_read_b64 %[u2], %[a2] offset:528\n"
      "ds_read_b64 %[t3], %[a3]\n"
      "ds_read_b64 %[u3], %[a3] offset:528\n"
      "s_waitcnt lgkmcnt(0)"
      : [t0] "=&v"(cur.lo[0]), [t1] "=&v"(cur.lo[1]), [t2] "=&v"(cur.lo[2]),
        [t3] "=&v"(cur.lo[3]), [u0] "=&v"(cur.hi[0]), [u1] "=&v"(cur.hi[1]),
        [u2] "=&v"(cur.hi[2]), [u3] "=&v"(cur.hi[3])
      : [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]), [a3] "v"(a[3]));
  ((rows_step<C, NSTEP, NK, PW>(lbase, tb, cur, addr, acc0, acc1),
    after(std::integral_constant<int, C>{})),
   ...);
}

#undef CPI_ROWS_READS
#undef CPI_ROWS_ADDRS
#undef CPI_ROWS_FMA
#undef CPI_ROWS_FMAS
#undef CPI_ROWS_ACC_OUT
#undef CPI_ROWS_FMA_IN
#undef CPI_ROWS_READ_OUT

// Copies of the first view's window in all phases (before the loop).
template <typename Load, typename Store, int... H>
__device__ __forceinline__ void rows_copy_all(Load&& load, Store&& store,
                                              std::integer_sequence<int, H...>) {
  ((load(std::integral_constant<int, H>{}), store(std::integral_constant<int, H>{})), ...);
}

template <int NA, int XR, int WW>
// (at least two waves per SIMD: the LDS of two work-groups fits a CU)
__global__ __launch_bounds__(NA * XR * 64 / rows_pairs_per_wave(NA * XR), 2) void k_ref_rows(
    const float* __restrict__ gamma, GeomI g, const int32_t* __restrict__ xe,
    const int2* __restrict__ yr, int groups, int tiles, int bands, int count,
    float* __restrict__ tout, int wout_pad) {
  typedef RowsShape<NA, XR, WW> Sh;
  constexpr int PW = Sh::PW;
  // two stages, each the window (WW columns of kRowsColStride floats) and
  // the view's table
  __shared__ __attribute__((aligned(16))) float ring[2 * Sh::STAGE];
  // All work-groups of one y_b on one XCD (work-groups go to the XCDs in
  // turn); within it the plane groups vary fastest, so the work-groups
  // resident on an XCD at one time read the same few column strips of each
  // view and keep them in its L2 even when they drift apart by many views.
  const int b = blockIdx.x;
  const int xcd = b & 7, local = b >> 3;
  const int per_yb = bands * tiles * groups;
  const int yb = xcd + 8 * (local / per_yb);
  if (yb >= g.hb) return;
  int rest = local % per_yb;
  const int gq = rest % groups;
  rest /= groups;
  const int t = rest % tiles;
  const int band = rest / tiles;
  const int r0 = band * kRowsBand;   // first view row of the band
  const int2 yrg = yr[int64_t(gq) * g.hb + yb];
  // a band with no touched row writes zeros and stops
  const bool band_live = r0 <= yrg.y && r0 + kRowsBand - 1 >= yrg.x;
  const int tid = threadIdx.x;
  const int ps = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int row = r0 + 2 * lane;     // this lane's rows: row, row + 1
  const int64_t pa = int64_t(g.wa) * g.ha;
  const float* vrow = gamma + int64_t(yb) * g.wb * pa;
  const int32_t* tab0 = xe + int64_t(gq * tiles + t) * g.wb * Sh::TAB;

  float acc0[PW], acc1[PW];
#pragma unroll
  for (int i = 0; i < PW; ++i) {
    acc0[i] = 0.0f;
    acc1[i] = 0.0f;
  }

  if (band_live) {
    // Copies: copy k of wave ps covers window rows 16 m .. 16 m + 15 and
    // columns 16 q .. 16 q + 15 (c = ps + k NPS, m = c % 8 = ps + NPS (k %
    // NM), q = c / 8 = k / NM); lane: row 16 m + lane / 4, columns
    // 16 q + 4 (lane % 4) ... + 3.  A view's copies run in PH phases of CPH
    // loads, spread over the pass of the previous view so that at most 8 are
    // held in registers.  Rows past the view repeat its last row.  (Element
    // offsets within a view: pa is below 2^31.)
    const int cr = lane >> 2, cc = 4 * (lane & 3);
    uint32_t roff[Sh::NM];
#pragma unroll
    for (int j = 0; j < Sh::NM; ++j) {
      const int r = r0 + 16 * (ps + Sh::NPS * j) + cr;
      roff[j] = uint32_t(((r < g.ha ? r : g.ha - 1) * g.wa + cc) * 4);
    }
    // Buffer loads (32-bit offsets from a per-view descriptor; a read past
    // the described range returns zero rather than touching memory).
    f4 win[Sh::CPH];
    f4 tab = f4{0.f, 0.f, 0.f, 0.f};
    int wx0_next = tab0[0];
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(tab0), short(0), int(g.wb * Sh::TAB * 4), kBufferWord3);
    auto load = [&](int xb, int wx0, auto phase) {
      constexpr int h = decltype(phase)::value;
      const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(vrow + int64_t(xb) * pa + wx0), short(0), int((pa - wx0) * 4),
          kBufferWord3);
#pragma unroll
      for (int i = 0; i < Sh::CPH; ++i) {
        const int k = h * Sh::CPH + i;
        win[i] = __builtin_bit_cast(
            f4, __builtin_amdgcn_raw_buffer_load_b128(vrs, roff[k % Sh::NM] + 64 * (k / Sh::NM),
                                                      0, 0));
      }
      if (h == Sh::PH - 1 && tid < Sh::TAB / 4)
        tab = __builtin_bit_cast(
            f4, __builtin_amdgcn_raw_buffer_load_b128(trs, (xb * Sh::TAB + 4 * tid) * 4, 0, 0));
    };
    auto store = [&](int stage, auto phase) {
      constexpr int h = decltype(phase)::value;
      float* st = ring + stage * Sh::STAGE;
#pragma unroll
      for (int i = 0; i < Sh::CPH; ++i) {
        const int k = h * Sh::CPH + i;
        const int m = ps + Sh::NPS * (k % Sh::NM), q = k / Sh::NM;
        float* d = st + (16 * q + cc) * kRowsColStride + 16 * m + cr;
        d[0] = win[i].x;
        d[kRowsColStride] = win[i].y;
        d[2 * kRowsColStride] = win[i].z;
        d[3 * kRowsColStride] = win[i].w;
      }
      if (h == Sh::PH - 1 && tid < Sh::TAB / 4)
        *reinterpret_cast<f4*>(st + Sh::WIN + 4 * tid) = tab;
    };

    rows_copy_all([&](auto ph) { load(0, wx0_next, ph); }, [&](auto ph) { store(0, ph); },
                  std::make_integer_sequence<int, Sh::PH>{});
    if (g.wb > 1) wx0_next = tab0[Sh::TAB];
    const uint32_t ring_base = uint32_t(reinterpret_cast<uintptr_t>(ring));
    // this lane's slot of the wave's table slice (offsets; w0 and w1 follow
    // at PW and 2 PW words)
    const uint32_t tab_lane = uint32_t((Sh::WIN + 4 + ps * 3 * PW + Sh::NK * (lane & 15)) * 4);
    for (int v = 0; v < g.wb; ++v) {
      // stage v & 1 holds view v; every wave is done with view v - 1's stage
      __syncthreads();
      const bool more = v + 1 < g.wb;
      const int wx1 = wx0_next;   // window start of view v + 1
      if (more) {
        load(v + 1, wx1, std::integral_constant<int, 0>{});
        if (v + 2 < g.wb) wx0_next = tab0[int64_t(v + 2) * Sh::TAB];
      }
      // the wave's pairs against view v; phase h of the next view's copies
      // is stored, and phase h + 1 loaded, after step NSTEP (h + 1) / PH - 1
      const uint32_t stage_base = ring_base + uint32_t((v & 1) * Sh::STAGE * 4);
      rows_view<Sh::NK, PW>(
          stage_base + tab_lane, stage_base + 8 * lane, acc0, acc1,
          [&](auto step) {
            constexpr int C = decltype(step)::value;
            constexpr int span = Sh::NSTEP / Sh::PH;
            if constexpr (Sh::PH > 1 && C < Sh::NSTEP - 1 && (C + 1) % span == 0) {
              constexpr int h = (C + 1) / span - 1;
              if (more) {
                store((v + 1) & 1, std::integral_constant<int, h>{});
                load(v + 1, wx1, std::integral_constant<int, h + 1>{});
              }
            }
          },
          std::make_integer_sequence<int, Sh::NSTEP>{});
      if (more) store((v + 1) & 1, std::integral_constant<int, Sh::PH - 1>{});
    }
  }

  const int64_t plane_stride = int64_t(g.hb) * g.ha * wout_pad;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = row + h;
    if (r >= g.ha) continue;
    const bool keep = band_live && r >= yrg.x && r <= yrg.y;
#pragma unroll
    for (int i = 0; i < PW; i += 4) {
      const int p = ps * PW + i;
      const int k = p / XR, j = p % XR;
      const int pl = gq * NA + k;
      if (pl < count) {
        const float* a = h ? acc1 : acc0;
        float4 w = keep ? make_float4(a[i], a[i + 1], a[i + 2], a[i + 3])
                        : make_float4(0.f, 0.f, 0.f, 0.f);
        float* d = tout + int64_t(pl) * plane_stride + (int64_t(yb) * g.ha + r) * wout_pad +
                   t * XR + j;
        *reinterpret_cast<float4*>(d) = w;
      }
    }
  }
}

// out(plane, y_r, x_r) = sum over y_b of wy0 * T(yc) + wy1 * T(yc + 1).
__global__ __launch_bounds__(256) void k_ref_rows_fold(GeomI g, const YEntry* __restrict__ ytab,
                                                       const float* __restrict__ tin,
                                                       int wout_pad, int first, int count,
                                                       float* __restrict__ out) {
  const int64_t opix = int64_t(g.out_w) * g.out_h;
  const int64_t n = opix * count;
  const int64_t plane_stride = int64_t(g.hb) * g.ha * wout_pad;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * 256) {
    const int pl = int(i / opix);
    const int64_t pix = i % opix;
    const int yr_ = int(pix / g.out_w), xr = int(pix % g.out_w);
    const YEntry* ye = ytab + int64_t(first + pl) * g.hb * g.out_h + yr_;
    const float* tp = tin + int64_t(pl) * plane_stride + xr;
    float acc = 0.0f;
    // 8 lens-plane rows' loads in flight at a time; summed in order of y_b
    int yb = 0;
    for (; yb + 8 <= g.hb; yb += 8) {
      float v0[8], v1[8], w0[8], w1[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const YEntry e = ye[int64_t(yb + k) * g.out_h];
        const float* r = tp + (int64_t(yb + k) * g.ha + e.row) * wout_pad;
        v0[k] = r[0];
        v1[k] = r[wout_pad];
        w0[k] = e.w0;
        w1[k] = e.w1;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += __builtin_fmaf(w1[k], v1[k], w0[k] * v0[k]);
    }
    for (; yb < g.hb; ++yb) {
      const YEntry e = ye[int64_t(yb) * g.out_h];
      const float* r = tp + (int64_t(yb) * g.ha + e.row) * wout_pad;
      acc += __builtin_fmaf(e.w1, r[wout_pad], e.w0 * r[0]);
    }
    out[int64_t(first + pl) * opix + pix] = acc;
  }
}

}  // namespace

bool rows_config_built(int na, int xr) {
  return (na == 8 && xr == 8) || (na == 4 && xr == 16) || (na == 8 && xr == 16) ||
         (na == 16 && xr == 8) || (na == 16 && xr == 16) || (na == 8 && xr == 32);
}

int rows_window_width(const RefGeom& g, const double* alphas, int n_alpha, int na, int xr) {
  // For each plane group, tile and lens-plane column, the sample coordinate
  // u = alpha (x_r - ca_x) + ca_x + (1 - alpha) mag_x (x_b - cb_x) is
  // bilinear in (alpha, x_r), so its range over the group's pairs lies
  // between its values at the four corners (alpha_min or alpha_max, first or
  // last column of the tile).  The cells span floor(u_max) - floor(u_min)
  // columns, plus the cell's second column, plus one column on each side for
  // the rounding of the coordinate's fraction.
  const int tiles = (g.out_w + xr - 1) / xr;
  int need = 0;
  for (int g0 = 0; g0 < n_alpha; g0 += na) {
    double lo = alphas[g0], hi = alphas[g0];
    for (int k = g0; k < n_alpha && k < g0 + na; ++k) {
      lo = std::fmin(lo, alphas[k]);
      hi = std::fmax(hi, alphas[k]);
    }
    for (int t = 0; t < tiles; ++t) {
      const double x0 = t * xr, x1 = std::fmin(t * xr + xr - 1, g.out_w - 1);
      for (int xb = 0; xb < g.wb; ++xb) {
        const double sb = g.mag_x * (xb - g.cb_x);
        double umin = 1e300, umax = -1e300;
        for (double a : {lo, hi})
          for (double x : {x0, x1}) {
            const double u = a * (x - g.ca_x) + g.ca_x + (1.0 - a) * sb;
            umin = std::fmin(umin, u);
            umax = std::fmax(umax, u);
          }
        const int w = int(std::floor(umax) - std::floor(umin)) + 4;
        if (w > need) need = w;
      }
    }
  }
  for (int ww : {16, 32, 64})
    if (need <= ww && g.wa >= ww) return ww;
  return 0;
}

template <int NA, int XR, int WW>
hipError_t launch_rows_ww(const float* gamma, const GeomI& gi, const int32_t* itab,
                          const float* ftab, const YEntry* ytab, int64_t stride, int n_alpha,
                          const RowsWorkspace& w, float* out, hipStream_t s) {
  const int tiles = (gi.out_w + XR - 1) / XR;
  const int wout_pad = tiles * XR;
  const int bands = (gi.ha + kRowsBand - 1) / kRowsBand;
  if (int64_t(wout_pad) > w.wout_cap) return hipErrorInvalidValue;
  for (int first = 0; first < n_alpha; first += w.chunk) {
    const int count = n_alpha - first < w.chunk ? n_alpha - first : w.chunk;
    const int groups = (count + NA - 1) / NA;
    const int64_t nx = int64_t(groups) * tiles * gi.wb;
    hipLaunchKernelGGL((k_rows_xtab<NA, XR>), dim3(unsigned(nx)), dim3(NA * XR), 0, s, gi, itab,
                       ftab, stride, first, count, tiles, WW, w.xe);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rows_yrange, dim3(unsigned(int64_t(groups) * gi.hb)), dim3(256), 0, s,
                       gi, ytab, first, count, NA, w.yr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nwg = int64_t(8) * ((gi.hb + 7) / 8) * bands * tiles * groups;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ref_rows<NA, XR, WW>), dim3(unsigned(nwg)),
                       dim3(RowsShape<NA, XR, WW>::NPS * 64), 0, s, gamma,
                       gi, w.xe, w.yr, groups, tiles, bands, count, w.t, wout_pad);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nf = int64_t(gi.out_w) * gi.out_h * count;
    int64_t gf = (nf + 255) / 256;
    if (gf > 65536) gf = 65536;
    hipLaunchKernelGGL(k_ref_rows_fold, dim3(unsigned(gf)), dim3(256), 0, s, gi, ytab, w.t,
                       wout_pad, first, count, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NA, int XR>
hipError_t launch_rows(int ww, const float* gamma, const GeomI& gi, const int32_t* itab,
                       const float* ftab, const YEntry* ytab, int64_t stride, int n_alpha,
                       const RowsWorkspace& w, float* out, hipStream_t s) {
  if (ww == 16)
    return launch_rows_ww<NA, XR, 16>(gamma, gi, itab, ftab, ytab, stride, n_alpha, w, out, s);
  if (ww == 32)
    return launch_rows_ww<NA, XR, 32>(gamma, gi, itab, ftab, ytab, stride, n_alpha, w, out, s);
  if (ww == 64)
    return launch_rows_ww<NA, XR, 64>(gamma, gi, itab, ftab, ytab, stride, n_alpha, w, out, s);
  return hipErrorInvalidValue;
}

bool rows_supported(const RefGeom& g, const double* alphas, int n_alpha, int na, int xr,
                    int64_t chunk) {
  if (!rows_config_built(na, xr) || chunk < 16 || chunk % 16 != 0 || g.wa < 2 || g.ha < 2)
    return false;
  return rows_window_width(g, alphas, n_alpha, na, xr) != 0;
}

hipError_t refocus_rows(const float* gamma, const RefGeom& g, const double* alphas,
                        const int32_t* itab, const float* ftab, const void* ytab, int64_t stride,
                        int n_alpha, int na, int xr, const RowsWorkspace& w, float* out,
                        hipStream_t s) {
  if (!rows_supported(g, alphas, n_alpha, na, xr, w.chunk)) return hipErrorInvalidValue;
  const int ww = rows_window_width(g, alphas, n_alpha, na, xr);
  const GeomI gi{g.wa, g.ha, g.wb, g.hb, g.out_w, g.out_h};
  const YEntry* yt = static_cast<const YEntry*>(ytab);
#define CPI_ROWS_CASE(NA_, XR_)                                                                \
  if (na == NA_ && xr == XR_)                                                                  \
    return launch_rows<NA_, XR_>(ww, gamma, gi, itab, ftab, yt, stride, n_alpha, w, out, s);
  CPI_ROWS_CASE(8, 8)
  CPI_ROWS_CASE(4, 16)
  CPI_ROWS_CASE(8, 16)
  CPI_ROWS_CASE(16, 8)
  CPI_ROWS_CASE(16, 16)
  CPI_ROWS_CASE(8, 32)
#undef CPI_ROWS_CASE
  return hipErrorInvalidValue;
}

}  // namespace cpi
