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
// lane: cells and weights come from a table (k_rows_xtab) through scalar
// loads, and the weights are scalar operands of the multiply-adds.  For
// every view x_b the work-group stages a window of the band's rows and WW
// columns (the union of its pairs' cells) in LDS, two stages deep, stored
// column by column: one ds_read2_b64 then gives a lane both taps of both its
// rows.  The window is loaded with coalesced 16-byte reads (16 rows x 64
// bytes per instruction) into registers while the previous view is
// interpolated, and stored transposed; a column stride of 132 floats keeps
// those stores free of bank conflicts.  Work-groups are mapped so that all
// those of one y_b run on one XCD and share its L2.
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
  int32_t* e = xe + idx * (4 + 3 * P);
  e[4 + p] = rel * kRowsColStride * 4;
  e[4 + P + p] = __builtin_bit_cast(int32_t, live ? w0 : 0.0f);
  e[4 + 2 * P + p] = __builtin_bit_cast(int32_t, live ? w1 : 0.0f);
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
  static constexpr int NPS = P / 64;              // waves (64 pairs each)
  static constexpr int TAB = 4 + 3 * P;           // table words per view (header, offsets, w0, w1)
  static constexpr int WIN = WW * kRowsColStride;    // window floats per stage
  static constexpr int STAGE = WIN + TAB;         // floats per stage
  static constexpr int NCP = 2 * (WW / 4);        // 16-row x 64-byte copies per view
  static constexpr int CPW = NCP / NPS;           // copies per wave per view
  static_assert(P % 64 == 0 && P <= 256 && (XR % 64 == 0 || 64 % XR == 0) && XR % 4 == 0,
                "pair layout");
  static_assert(WW == 16 || WW == 32 || WW == 64, "window width");
  static_assert(NCP % NPS == 0, "copies per wave");
  static_assert(TAB / 4 <= NPS * 64, "table copy");
  static_assert(2 * STAGE * 4 <= 160 * 1024, "LDS");
};

typedef int i4 __attribute__((ext_vector_type(4)));

// A wave's pass over its 64 pairs for one view, 4 pairs (chunk C) per step.
// Each step is one inline-asm block that issues the LDS reads of chunk C + 1
// (the 8 tap reads: both rows of a lane at the cell's column and at the next,
// single 8-byte reads, which run at twice the rate of the paired form the
// compiler would merge them into; the weights of chunk C + 1 and the cell
// offsets of chunk C + 2, broadcast reads of the staged table at `tb`:
// offsets, then P w0, then P w1), then the 16 multiply-adds of chunk C on
// values read by the previous step, then waits for its reads: the LDS
// latency of one chunk overlaps the arithmetic of the previous one.
struct RowsChunk {
  f2 lo[4], hi[4];   // taps: rows 2 lane, 2 lane + 1 at the cell's column / the next
  f4 w0, w1;         // weights of the 4 pairs
};

template <int C, int P>
__device__ __forceinline__ void rows_step(uint32_t tb, uint32_t lbase, RowsChunk& cur,
                                          i4& off_next, float (&acc0)[64], float (&acc1)[64]) {
  static_assert(kRowsColStride * 4 == 528, "column offset below");
  constexpr int p = 4 * C;
  if constexpr (C == 15) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float w0 = cur.w0[i], w1 = cur.w1[i];
      acc0[p + i] = __builtin_fmaf(w0, cur.lo[i].x, acc0[p + i]);
      acc1[p + i] = __builtin_fmaf(w0, cur.lo[i].y, acc1[p + i]);
      acc0[p + i] = __builtin_fmaf(w1, cur.hi[i].x, acc0[p + i]);
      acc1[p + i] = __builtin_fmaf(w1, cur.hi[i].y, acc1[p + i]);
    }
  } else {
    constexpr int kW0 = P * 4 + 16 * (C + 1), kW1 = 2 * P * 4 + 16 * (C + 1);
    constexpr int kOn = 16 * (C + 2 < 16 ? C + 2 : 15);
    const uint32_t a0 = lbase + uint32_t(off_next.x), a1 = lbase + uint32_t(off_next.y);
    const uint32_t a2 = lbase + uint32_t(off_next.z), a3 = lbase + uint32_t(off_next.w);
    RowsChunk nx;
    i4 on;
    asm volatile(
        "ds_read_b64 %[t0], %[a0]\n"
        "ds_read_b64 %[u0], %[a0] offset:528\n"
        "ds_read_b64 %[t1], %[a1]\n"
        "ds_read_b64 %[u1], %[a1] offset:528\n"
        "ds_read_b64 %[t2], %[a2]\n"
        "ds_read_b64 %[u2], %[a2] offset:528\n"
        "ds_read_b64 %[t3], %[a3]\n"
        "ds_read_b64 %[u3], %[a3] offset:528\n"
        "ds_read_b128 %[w0], %[tb] offset:%[kw0]\n"
        "ds_read_b128 %[w1], %[tb] offset:%[kw1]\n"
        "ds_read_b128 %[on], %[tb] offset:%[kon]\n"
        "v_fmac_f32 %[c00], %[x0], %[l0x]\n"
        "v_fmac_f32 %[c10], %[x0], %[l0y]\n"
        "v_fmac_f32 %[c00], %[y0], %[h0x]\n"
        "v_fmac_f32 %[c10], %[y0], %[h0y]\n"
        "v_fmac_f32 %[c01], %[x1], %[l1x]\n"
        "v_fmac_f32 %[c11], %[x1], %[l1y]\n"
        "v_fmac_f32 %[c01], %[y1], %[h1x]\n"
        "v_fmac_f32 %[c11], %[y1], %[h1y]\n"
        "v_fmac_f32 %[c02], %[x2], %[l2x]\n"
        "v_fmac_f32 %[c12], %[x2], %[l2y]\n"
        "v_fmac_f32 %[c02], %[y2], %[h2x]\n"
        "v_fmac_f32 %[c12], %[y2], %[h2y]\n"
        "v_fmac_f32 %[c03], %[x3], %[l3x]\n"
        "v_fmac_f32 %[c13], %[x3], %[l3y]\n"
        "v_fmac_f32 %[c03], %[y3], %[h3x]\n"
        "v_fmac_f32 %[c13], %[y3], %[h3y]\n"
        "s_waitcnt lgkmcnt(0)"
        : [t0] "=&v"(nx.lo[0]), [t1] "=&v"(nx.lo[1]), [t2] "=&v"(nx.lo[2]), [t3] "=&v"(nx.lo[3]),
          [u0] "=&v"(nx.hi[0]), [u1] "=&v"(nx.hi[1]), [u2] "=&v"(nx.hi[2]), [u3] "=&v"(nx.hi[3]),
          [w0] "=&v"(nx.w0), [w1] "=&v"(nx.w1), [on] "=&v"(on),
          [c00] "+v"(acc0[p]), [c01] "+v"(acc0[p + 1]), [c02] "+v"(acc0[p + 2]),
          [c03] "+v"(acc0[p + 3]), [c10] "+v"(acc1[p]), [c11] "+v"(acc1[p + 1]),
          [c12] "+v"(acc1[p + 2]), [c13] "+v"(acc1[p + 3])
        : [a0] "v"(a0), [a1] "v"(a1), [a2] "v"(a2), [a3] "v"(a3), [tb] "v"(tb),
          [kw0] "i"(kW0), [kw1] "i"(kW1), [kon] "i"(kOn),
          [x0] "v"(cur.w0.x), [x1] "v"(cur.w0.y), [x2] "v"(cur.w0.z), [x3] "v"(cur.w0.w),
          [y0] "v"(cur.w1.x), [y1] "v"(cur.w1.y), [y2] "v"(cur.w1.z), [y3] "v"(cur.w1.w),
          [l0x] "v"(cur.lo[0].x), [l0y] "v"(cur.lo[0].y), [l1x] "v"(cur.lo[1].x),
          [l1y] "v"(cur.lo[1].y), [l2x] "v"(cur.lo[2].x), [l2y] "v"(cur.lo[2].y),
          [l3x] "v"(cur.lo[3].x), [l3y] "v"(cur.lo[3].y), [h0x] "v"(cur.hi[0].x),
          [h0y] "v"(cur.hi[0].y), [h1x] "v"(cur.hi[1].x), [h1y] "v"(cur.hi[1].y),
          [h2x] "v"(cur.hi[2].x), [h2y] "v"(cur.hi[2].y), [h3x] "v"(cur.hi[3].x),
          [h3y] "v"(cur.hi[3].y));
    cur = nx;
    off_next = on;
  }
}

template <int P, int... C>
__device__ __forceinline__ void rows_view(uint32_t tb, uint32_t lbase, float (&acc0)[64],
                                          float (&acc1)[64], std::integer_sequence<int, C...>) {
  // chunk 0's cells, then its taps and weights and chunk 1's cells
  i4 off0, off1;
  RowsChunk cur;
  asm volatile("ds_read_b128 %0, %1\n"
               "s_waitcnt lgkmcnt(0)"
               : "=&v"(off0)
               : "v"(tb));
  {
    const uint32_t a0 = lbase + uint32_t(off0.x), a1 = lbase + uint32_t(off0.y);
    const uint32_t a2 = lbase + uint32_t(off0.z), a3 = lbase + uint32_t(off0.w);
    asm volatile(
        "ds_read_b64 %[t0], %[a0]\n"
        "ds_read_b64 %[u0], %[a0] offset:528\n"
        "ds_read_b64 %[t1], %[a1]\n"
        "ds_read_b64 %[u1], %[a1] offset:528\n"
        "ds_read_b64 %[t2], %[a2]\n"
        "ds_read_b64 %[u2], %[a2] offset:528\n"
        "ds_read_b64 %[t3], %[a3]\n"
        "ds_read_b64 %[u3], %[a3] offset:528\n"
        "ds_read_b128 %[w0], %[tb] offset:%[kw0]\n"
        "ds_read_b128 %[w1], %[tb] offset:%[kw1]\n"
        "ds_read_b128 %[on], %[tb] offset:16\n"
        "s_waitcnt lgkmcnt(0)"
        : [t0] "=&v"(cur.lo[0]), [t1] "=&v"(cur.lo[1]), [t2] "=&v"(cur.lo[2]),
          [t3] "=&v"(cur.lo[3]), [u0] "=&v"(cur.hi[0]), [u1] "=&v"(cur.hi[1]),
          [u2] "=&v"(cur.hi[2]), [u3] "=&v"(cur.hi[3]), [w0] "=&v"(cur.w0),
          [w1] "=&v"(cur.w1), [on] "=&v"(off1)
        : [a0] "v"(a0), [a1] "v"(a1), [a2] "v"(a2), [a3] "v"(a3), [tb] "v"(tb),
          [kw0] "i"(P * 4), [kw1] "i"(2 * P * 4));
  }
  (rows_step<C, P>(tb, lbase, cur, off1, acc0, acc1), ...);
}

template <int NA, int XR, int WW>
// (at least two waves per SIMD: the LDS of two work-groups fits a CU)
__global__ __launch_bounds__(NA * XR, 2) void k_ref_rows(
    const float* __restrict__ gamma, GeomI g, const int32_t* __restrict__ xe,
    const int2* __restrict__ yr, int groups, int tiles, int bands, int count,
    float* __restrict__ tout, int wout_pad) {
  typedef RowsShape<NA, XR, WW> Sh;
  constexpr int P = Sh::P;
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

  float acc0[64], acc1[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    acc0[i] = 0.0f;
    acc1[i] = 0.0f;
  }

  if (band_live) {
    // Copies: instruction k of wave ps covers window rows 16 m .. 16 m + 15
    // and columns 16 q .. 16 q + 15 (m = c % 8, q = c / 8, c = ps + k NPS);
    // lane: row 16 m + lane / 4, columns 16 q + 4 (lane % 4) ... + 3.  The
    // window start of a view comes through a scalar load one view ahead.
    const int cr = lane >> 2, cc = 4 * (lane & 3);
    // Every block of the band is copied (straight-line loads, so that they
    // are all in flight together); rows past the view repeat its last row.
    // (element offsets within a view: pa is below 2^31)
    uint32_t roff[Sh::CPW];
#pragma unroll
    for (int k = 0; k < Sh::CPW; ++k) {
      const int c = ps + k * Sh::NPS;
      const int r = r0 + 16 * (c & 7) + cr;
      roff[k] = uint32_t((r < g.ha ? r : g.ha - 1) * g.wa + 16 * (c >> 3) + cc);
    }
    // Buffer loads (32-bit offsets from a per-view descriptor; a read past
    // the described range returns zero rather than touching memory).
    f4 win[Sh::CPW];
    f4 tab = f4{0.f, 0.f, 0.f, 0.f};
    int wx0_next = tab0[0];
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(tab0), short(0), int(g.wb * Sh::TAB * 4), kBufferWord3);
    auto load = [&](int xb, int wx0) {
      const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(vrow + int64_t(xb) * pa + wx0), short(0), int((pa - wx0) * 4),
          kBufferWord3);
#pragma unroll
      for (int k = 0; k < Sh::CPW; ++k)
        win[k] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(vrs, roff[k] * 4, 0, 0));
      if (tid < Sh::TAB / 4)
        tab = __builtin_bit_cast(
            f4, __builtin_amdgcn_raw_buffer_load_b128(trs, (xb * Sh::TAB + 4 * tid) * 4, 0, 0));
    };
    auto store = [&](int stage) {
      float* st = ring + stage * Sh::STAGE;
#pragma unroll
      for (int k = 0; k < Sh::CPW; ++k) {
        const int c = ps + k * Sh::NPS;
        float* d = st + (16 * (c >> 3) + cc) * kRowsColStride + 16 * (c & 7) + cr;
        d[0] = win[k].x;
        d[kRowsColStride] = win[k].y;
        d[2 * kRowsColStride] = win[k].z;
        d[3 * kRowsColStride] = win[k].w;
      }
      if (tid < Sh::TAB / 4)
        *reinterpret_cast<f4*>(st + Sh::WIN + 4 * tid) = tab;
    };

    load(0, wx0_next);
    if (g.wb > 1) wx0_next = tab0[Sh::TAB];
    store(0);
    const uint32_t ring_base = uint32_t(reinterpret_cast<uintptr_t>(ring));
    for (int v = 0; v < g.wb; ++v) {
      // stage v & 1 holds view v; every wave is done with view v - 1's stage
      __syncthreads();
      if (v + 1 < g.wb) {
        load(v + 1, wx0_next);
        if (v + 2 < g.wb) wx0_next = tab0[int64_t(v + 2) * Sh::TAB];
      }
      // the wave's 64 pairs against view v: table at tb (offsets, w0, w1 of
      // its pairs), window columns at lbase (this lane's two rows)
      const uint32_t stage_base = ring_base + uint32_t((v & 1) * Sh::STAGE * 4);
      rows_view<P>(stage_base + uint32_t((Sh::WIN + 4 + ps * 64) * 4), stage_base + 8 * lane,
                   acc0, acc1, std::make_integer_sequence<int, 16>{});
      if (v + 1 < g.wb) store((v + 1) & 1);
    }
  }

  const int64_t plane_stride = int64_t(g.hb) * g.ha * wout_pad;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = row + h;
    if (r >= g.ha) continue;
    const bool keep = band_live && r >= yrg.x && r <= yrg.y;
#pragma unroll
    for (int i = 0; i < 64; i += 4) {
      const int p = ps * 64 + i;
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
    hipLaunchKernelGGL((k_ref_rows<NA, XR, WW>), dim3(unsigned(nwg)), dim3(NA * XR), 0, s, gamma,
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
