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
// x pass (k_ref_rows).  A work-group owns one lens-plane row y_b, a group of
// NA planes and XR consecutive output columns: P = NA * XR (plane, column)
// pairs.  Its lanes are view rows, so for a given view and pair the column
// cell is the same for every lane: cells and weights come from a table
// (k_rows_xtab) through scalar loads, the weights are scalar operands of the
// multiply-adds, and each lane reads its own row's two taps from LDS (one
// ds_read2_b32).  For every view x_b the work-group stages a window of
// all view rows and WW columns (the union of its pairs' cells) in LDS with
// direct global->LDS copies, two stages deep; window rows sit in blocks of
// 64 floats plus one pad float, so the 64 lanes of a wave, reading one
// column of 64 consecutive rows, hit 64 distinct banks.  Work-groups are
// mapped so that all those of one y_b run on one XCD and share its L2.
//
// Fold pass (k_ref_rows_fold): one thread per output pixel of a plane sums
// the two T rows of each y_b with the row weights.
//
// Planes are processed in chunks whose T fits the caller's workspace.  Both
// sums run in a fixed order (x_b, then y_b), so results are bitwise
// reproducible for a given configuration.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"
#include "refocus_common.h"

namespace cpi {

namespace {

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

struct RowsHead {
  int wx0;         // first window column of the view for this (group, tile)
  uint32_t live;   // bit c: some pair in 16-pair chunk c has a nonzero weight
                   // (a wave takes its 64 pairs 32 at a time, skipping a
                   // half whose two chunks are both dead)
};

// Column cells of every (plane, output column) pair of work-group (group gq,
// tile t) against lens-plane column x_b: window start, and per pair the
// column of its cell in the window row and its two weights (zero for pairs
// past the planes or columns, or whose taps fall outside the view).  One
// block per (gq, t, x_b), one thread per pair.  The arithmetic is that of the
// other refocus kernels.
template <int NA, int XR>
__global__ __launch_bounds__(NA * XR) void k_rows_xtab(GeomI g, const int32_t* __restrict__ itab,
                                                     const float* __restrict__ ftab,
                                                     int64_t stride, int first, int count,
                                                     int tiles, int ww, RowsHead* __restrict__ head,
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
    atomicOr(&slive, 1u << (p / 16));
  }
  __syncthreads();
  int wx0 = slive ? smin : 0;
  if (wx0 > g.wa - ww) wx0 = g.wa - ww;
  if (wx0 < 0) wx0 = 0;
  // The host's window bound keeps every cell in the window; the clamp keeps
  // LDS reads inside it regardless.
  int rel = live ? c - wx0 : 0;
  rel = rel < 0 ? 0 : (rel > ww - 2 ? ww - 2 : rel);
  int32_t* e = xe + idx * 3 * P;
  e[p] = rel;
  e[P + p] = __builtin_bit_cast(int32_t, live ? w0 : 0.0f);
  e[2 * P + p] = __builtin_bit_cast(int32_t, live ? w1 : 0.0f);
  if (p == 0) head[idx] = RowsHead{wx0, slive};
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

template <int NA, int XR, int NWV, int WW>
struct RowsShape {
  static constexpr int P = NA * XR;               // (plane, column) pairs
  static constexpr int NPS = P / 64;              // pair sets (waves along the pairs)
  static constexpr int NWAVES = NWV * NPS;
  static constexpr int RS = WW + 1;               // LDS row stride (odd: conflict-free columns)
  static constexpr int TAB = 3 * P;               // table words per view (offsets, w0, w1)
  static constexpr int STAGE = 64 * NWV * RS + TAB;   // floats per stage
  static constexpr int LPL = WW / 4 / NPS;        // 16-byte window loads per lane per view
  static_assert(P % 64 == 0 && (XR % 64 == 0 || 64 % XR == 0) && XR % 4 == 0, "pair layout");
  static_assert(WW == 16 || WW == 32 || WW == 64, "window width");
  static_assert((WW / 4) % NPS == 0, "window loads per wave");
  static_assert(NWAVES * 64 <= 1024 && TAB / 4 <= NWAVES * 64, "work-group size");
  static_assert(2 * STAGE * 4 <= 160 * 1024, "LDS");
};

// (NWV * NA * XR threads: NWV row waves for each set of 64 pairs)
template <int NA, int XR, int NWV, int WW>
__global__ __launch_bounds__(NWV * NA * XR) void k_ref_rows(
    const float* __restrict__ gamma, GeomI g, const RowsHead* __restrict__ head,
    const int32_t* __restrict__ xe, const int2* __restrict__ yr, int groups, int tiles, int count,
    float* __restrict__ tout, int wout_pad) {
  typedef RowsShape<NA, XR, NWV, WW> Sh;
  constexpr int P = Sh::P;
  // two stages, each the window (64 NWV rows of RS floats) and the view's
  // table (offsets, w0, w1 of the P pairs)
  __shared__ __attribute__((aligned(16))) float ring[2 * Sh::STAGE];
  // All work-groups of one y_b on one XCD (work-groups go to the XCDs in
  // turn), and within it the plane groups fastest: the work-groups resident
  // on an XCD at one time cover all plane groups of a few adjacent tiles, so
  // the views' column strips they read stay in its L2 even when they drift
  // apart by many views.
  const int b = blockIdx.x;
  const int xcd = b & 7, local = b >> 3;
  const int gt = groups * tiles;
  const int yb = xcd + 8 * (local / gt);
  if (yb >= g.hb) return;
  const int rest = local % gt;
  const int t = rest / groups, gq = rest % groups;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int ps = wave / NWV, rb = wave % NWV;
  const int row = rb * 64 + lane;
  const int2 yrg = yr[int64_t(gq) * g.hb + yb];
  const bool wave_live = rb * 64 <= yrg.y && rb * 64 + 63 >= yrg.x && rb * 64 < g.ha;
  const bool row_live = row < g.ha && row >= yrg.x && row <= yrg.y;
  const int64_t pa = int64_t(g.wa) * g.ha;
  const float* vrow = gamma + int64_t(yb) * g.wb * pa;
  const int64_t hidx0 = int64_t(gq * tiles + t) * g.wb;

  // Next view's window (this lane's row, its share of the 16-byte chunks)
  // and table piece, loaded into registers while the current view is
  // interpolated, then stored to the other stage.
  f4u win[Sh::LPL];
  float4 tab = make_float4(0.f, 0.f, 0.f, 0.f);
  uint32_t live_next = 0u;
  auto load = [&](int xb) {
    const RowsHead h = head[hidx0 + xb];
    live_next = h.live;
    const float* src = vrow + int64_t(xb) * pa + int64_t(row) * g.wa + h.wx0;
#pragma unroll
    for (int i = 0; i < Sh::LPL; ++i) {
      const int c = ps + i * Sh::NPS;   // chunk of 4 columns (4-byte aligned)
      if (row_live) win[i] = *reinterpret_cast<const f4u*>(src + 4 * c);
    }
    if (tid < Sh::TAB / 4)
      tab = *reinterpret_cast<const float4*>(xe + (hidx0 + xb) * Sh::TAB + 4 * tid);
  };
  auto store = [&](int stage) {
    float* st = ring + stage * Sh::STAGE;
    float* rp = st + row * Sh::RS;
#pragma unroll
    for (int i = 0; i < Sh::LPL; ++i) {
      const int c = ps + i * Sh::NPS;
      if (row_live) {
        rp[4 * c] = win[i].x;
        rp[4 * c + 1] = win[i].y;
        rp[4 * c + 2] = win[i].z;
        rp[4 * c + 3] = win[i].w;
      }
    }
    if (tid < Sh::TAB / 4)
      *reinterpret_cast<float4*>(st + 64 * NWV * Sh::RS + 4 * tid) = tab;
  };

  float acc[64];
#pragma unroll
  for (int i = 0; i < 64; ++i) acc[i] = 0.0f;

  load(0);
  store(0);
  uint32_t live = live_next;
  for (int v = 0; v < g.wb; ++v) {
    // stage v & 1 holds view v; every wave is done with view v - 1's stage
    __syncthreads();
    if (v + 1 < g.wb) load(v + 1);
    if (wave_live) {
      const float* st = ring + (v & 1) * Sh::STAGE;
      const float* rp = st + row * Sh::RS;
      const int32_t* to = reinterpret_cast<const int32_t*>(st + 64 * NWV * Sh::RS) + ps * 64;
      const float* tw0 = st + 64 * NWV * Sh::RS + P + ps * 64;
      const float* tw1 = tw0 + P;
      // 16 pairs at a time: cells and weights as broadcast LDS reads, then
      // every tap read before the first multiply-add uses one
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if ((live >> (ps * 4 + c)) & 1u) {
          float t0[16], t1[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const float* q = rp + to[c * 16 + i];
            t0[i] = q[0];
            t1[i] = q[1];
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            acc[c * 16 + i] = __builtin_fmaf(tw0[c * 16 + i], t0[i], acc[c * 16 + i]);
            acc[c * 16 + i] = __builtin_fmaf(tw1[c * 16 + i], t1[i], acc[c * 16 + i]);
          }
        }
      }
    }
    if (v + 1 < g.wb) store((v + 1) & 1);
    live = live_next;
  }

  if (row >= g.ha) return;
  const int64_t plane_stride = int64_t(g.hb) * g.ha * wout_pad;
#pragma unroll
  for (int i = 0; i < 64; i += 4) {
    const int p = ps * 64 + i;
    const int k = p / XR, j = p % XR;
    const int pl = gq * NA + k;
    if (pl < count) {
      float4 w = (wave_live && row_live)
                     ? make_float4(acc[i], acc[i + 1], acc[i + 2], acc[i + 3])
                     : make_float4(0.f, 0.f, 0.f, 0.f);
      float* d = tout + int64_t(pl) * plane_stride + (int64_t(yb) * g.ha + row) * wout_pad +
                 t * XR + j;
      *reinterpret_cast<float4*>(d) = w;
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
    for (int yb = 0; yb < g.hb; ++yb) {
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
         (na == 16 && xr == 16) || (na == 8 && xr == 32);
}

int rows_window_width(const RefGeom& g, const double* alphas, int n_alpha, int na, int xr) {
  const double ax = std::fmax(std::fabs(g.ca_x), std::fabs(g.out_w - 1 - g.ca_x));
  const double bx = std::fmax(std::fabs(g.cb_x), std::fabs(g.wb - 1 - g.cb_x));
  double need = 0.0;
  for (int g0 = 0; g0 < n_alpha; g0 += na) {
    double lo = alphas[g0], hi = alphas[g0], am = 0.0;
    for (int k = g0; k < n_alpha && k < g0 + na; ++k) {
      lo = std::fmin(lo, alphas[k]);
      hi = std::fmax(hi, alphas[k]);
      am = std::fmax(am, std::fabs(alphas[k]));
    }
    // the range of the sample coordinate over the group's pairs at any x_b,
    // plus the cell's second column and one column on each side for the
    // rounding of the coordinate's fraction
    need = std::fmax(need, am * (xr - 1) + (hi - lo) * (ax + std::fabs(g.mag_x) * bx) + 5.0);
  }
  for (int ww : {16, 32, 64})
    if (need <= ww && g.wa >= ww) return ww;
  return 0;
}

template <int NA, int XR, int NWV, int WW>
hipError_t launch_rows_ww(const float* gamma, const GeomI& gi, const int32_t* itab,
                          const float* ftab, const YEntry* ytab, int64_t stride, int n_alpha,
                          const RowsWorkspace& w, float* out, hipStream_t s) {
  typedef RowsShape<NA, XR, NWV, WW> Sh;
  const int tiles = (gi.out_w + XR - 1) / XR;
  const int wout_pad = tiles * XR;
  if (int64_t(wout_pad) > w.wout_cap) return hipErrorInvalidValue;
  for (int first = 0; first < n_alpha; first += w.chunk) {
    const int count = n_alpha - first < w.chunk ? n_alpha - first : w.chunk;
    const int groups = (count + NA - 1) / NA;
    const int64_t nx = int64_t(groups) * tiles * gi.wb;
    hipLaunchKernelGGL((k_rows_xtab<NA, XR>), dim3(unsigned(nx)), dim3(NA * XR), 0, s, gi, itab,
                       ftab, stride, first, count, tiles, WW, static_cast<RowsHead*>(w.head), w.xe);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rows_yrange, dim3(unsigned(int64_t(groups) * gi.hb)), dim3(256), 0, s,
                       gi, ytab, first, count, NA, w.yr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nwg = int64_t(8) * ((gi.hb + 7) / 8) * groups * tiles;
    if (nwg > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ref_rows<NA, XR, NWV, WW>), dim3(unsigned(nwg)), dim3(Sh::NWAVES * 64),
                       0, s, gamma, gi, static_cast<const RowsHead*>(w.head), w.xe, w.yr, groups,
                       tiles, count, w.t, wout_pad);
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

template <int NA, int XR, int NWV>
hipError_t launch_rows_nwv(int ww, const float* gamma, const GeomI& gi, const int32_t* itab,
                           const float* ftab, const YEntry* ytab, int64_t stride, int n_alpha,
                           const RowsWorkspace& w, float* out, hipStream_t s) {
  if (ww == 16)
    return launch_rows_ww<NA, XR, NWV, 16>(gamma, gi, itab, ftab, ytab, stride, n_alpha, w, out,
                                           s);
  if (ww == 32)
    return launch_rows_ww<NA, XR, NWV, 32>(gamma, gi, itab, ftab, ytab, stride, n_alpha, w, out,
                                           s);
  if (ww == 64)
    return launch_rows_ww<NA, XR, NWV, 64>(gamma, gi, itab, ftab, ytab, stride, n_alpha, w, out,
                                           s);
  return hipErrorInvalidValue;
}

bool rows_supported(const RefGeom& g, const double* alphas, int n_alpha, int na, int xr,
                    int64_t chunk) {
  if (!rows_config_built(na, xr) || chunk < 16 || chunk % 16 != 0 || g.wa < 2 || g.ha < 2 ||
      g.ha > 256)
    return false;
  const int ww = rows_window_width(g, alphas, n_alpha, na, xr);
  return ww != 0 && g.ha % (64 / ww) == 0;
}

hipError_t refocus_rows(const float* gamma, const RefGeom& g, const double* alphas,
                        const int32_t* itab, const float* ftab, const void* ytab, int64_t stride,
                        int n_alpha, int na, int xr, const RowsWorkspace& w, float* out,
                        hipStream_t s) {
  if (!rows_supported(g, alphas, n_alpha, na, xr, w.chunk)) return hipErrorInvalidValue;
  const int ww = rows_window_width(g, alphas, n_alpha, na, xr);
  const int nwv = (g.ha + 63) / 64;
  const GeomI gi{g.wa, g.ha, g.wb, g.hb, g.out_w, g.out_h};
  const YEntry* yt = static_cast<const YEntry*>(ytab);
#define CPI_ROWS_CASE(NA_, XR_)                                                                \
  if (na == NA_ && xr == XR_) {                                                                \
    if (nwv == 1)                                                                              \
      return launch_rows_nwv<NA_, XR_, 1>(ww, gamma, gi, itab, ftab, yt, stride, n_alpha, w,   \
                                          out, s);                                             \
    if (nwv == 2)                                                                              \
      return launch_rows_nwv<NA_, XR_, 2>(ww, gamma, gi, itab, ftab, yt, stride, n_alpha, w,   \
                                          out, s);                                             \
    if (nwv <= 4)                                                                              \
      return launch_rows_nwv<NA_, XR_, 4>(ww, gamma, gi, itab, ftab, yt, stride, n_alpha, w,   \
                                          out, s);                                             \
  }
  CPI_ROWS_CASE(8, 8)
  CPI_ROWS_CASE(4, 16)
  CPI_ROWS_CASE(8, 16)
  CPI_ROWS_CASE(16, 16)
  CPI_ROWS_CASE(8, 32)
#undef CPI_ROWS_CASE
  return hipErrorInvalidValue;
}

}  // namespace cpi
