// Refocusing: shift-and-sum of the perspective views of Gamma.
//
// For plane alpha, output pixel (x_r, y_r) and detector-B pixel (x_b, y_b)
// the view Gamma(., rho_b) (Ha x Wa, view-major storage) is sampled
// bilinearly at
//     u_x = a_x(x_r) + b_x(x_b),  a_x = alpha*(x_r - ca_x) + ca_x,
//                                 b_x = (1 - alpha)*mag_x*(x_b - cb_x)
// (likewise in y) and the samples are summed over rho_b; corners outside the
// view contribute zero.  The interpolation points move with the plane, so
// they are computed on the fly from small per-plane tables (the paper builds
// them inside its refocusing kernel, Section 4.1): every a_x, a_y, b_x, b_y
// is formed in FP64 and split into an integer part and an FP32 fraction;
// the device adds the two parts of u and carries the fraction's overflow.
// The x tables depend on (plane, x_r) and (plane, x_b) only, the y tables on
// (plane, y_r) and (plane, y_b) only, so the per-sample cost is the four
// taps and their weights.
//
// Summation is blocked: samples are summed over x_b for one y_b, and those
// row sums are summed over y_b (and, for the batched kernels, over view-row
// splits in a fixed order), so the result is bitwise reproducible for a
// given configuration.  Three kernels evaluate the sum: k_ref_plain (one
// plane per launch, direct gathers), k_ref_batched (many planes per launch,
// each output row interpolating its view rows) and k_ref_sep (many planes
// per launch, column interpolants summed over x_b before the row weights).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "refocus_common.h"

namespace cpi {

namespace {

struct AlphaPack {
  double a[kAlphaPerLaunch];
};

__global__ __launch_bounds__(256) void k_ref_tables(AlphaPack ap, int count, int first,
                                                    RefGeom g, int64_t stride,
                                                    int32_t* __restrict__ itab,
                                                    float* __restrict__ ftab) {
  const int k = blockIdx.x;
  if (k >= count) return;
  const double alpha = ap.a[k];
  const int64_t base = int64_t(first + k) * stride;
  const int e_ay = g.out_w, e_bx = g.out_w + g.out_h, e_by = e_bx + g.wb;
  for (int64_t e = threadIdx.x; e < stride; e += blockDim.x) {
    double v;
    if (e < e_ay) {
      v = alpha * (double(e) - g.ca_x) + g.ca_x;
    } else if (e < e_bx) {
      v = alpha * (double(e - e_ay) - g.ca_y) + g.ca_y;
    } else if (e < e_by) {
      v = (1.0 - alpha) * g.mag_x * (double(e - e_bx) - g.cb_x);
    } else {
      v = (1.0 - alpha) * g.mag_y * (double(e - e_by) - g.cb_y);
    }
    const double fl = floor(v);
    int32_t iv = int32_t(fl);
    float f = float(v - fl);
    if (f >= 1.0f) {
      iv += 1;
      f = 0.0f;
    }
    itab[base + e] = iv;
    ftab[base + e] = f;
  }
}

__device__ __forceinline__ float tap(const float* __restrict__ view, int wa, int ha, int x,
                                     int y) {
  return (x >= 0 && x < wa && y >= 0 && y < ha) ? view[int64_t(y) * wa + x] : 0.0f;
}

// One thread per output pixel of one plane; direct gathers from Gamma.
__global__ __launch_bounds__(256) void k_ref_plain(const float* __restrict__ gamma, GeomI g,
                                                   const int32_t* __restrict__ itab,
                                                   const float* __restrict__ ftab,
                                                   int64_t stride, int plane,
                                                   float* __restrict__ out) {
  const int64_t opix = int64_t(g.out_w) * g.out_h;
  const int64_t pix = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (pix >= opix) return;
  const int xr = int(pix % g.out_w), yr = int(pix / g.out_w);
  const int32_t* it = itab + int64_t(plane) * stride;
  const float* ft = ftab + int64_t(plane) * stride;
  const int iax = it[xr], iay = it[g.out_w + yr];
  const float fax = ft[xr], fay = ft[g.out_w + yr];
  const int32_t* ibx = it + g.out_w + g.out_h;
  const float* fbx = ft + g.out_w + g.out_h;
  const int32_t* iby = ibx + g.wb;
  const float* fby = fbx + g.wb;
  const int64_t pa = int64_t(g.wa) * g.ha;
  float acc = 0.0f;
  for (int yb = 0; yb < g.hb; ++yb) {
    int y0 = iay + iby[yb];
    float fy = fay + fby[yb];
    if (fy >= 1.0f) {
      y0 += 1;
      fy -= 1.0f;
    }
    float row = 0.0f;
    for (int xb = 0; xb < g.wb; ++xb) {
      int x0 = iax + ibx[xb];
      float fx = fax + fbx[xb];
      if (fx >= 1.0f) {
        x0 += 1;
        fx -= 1.0f;
      }
      const float* view = gamma + (int64_t(yb) * g.wb + xb) * pa;
      const float g00 = tap(view, g.wa, g.ha, x0, y0);
      const float g01 = tap(view, g.wa, g.ha, x0 + 1, y0);
      const float g10 = tap(view, g.wa, g.ha, x0, y0 + 1);
      const float g11 = tap(view, g.wa, g.ha, x0 + 1, y0 + 1);
      const float top = (1.0f - fx) * g00 + fx * g01;
      const float bot = (1.0f - fx) * g10 + fx * g11;
      row += (1.0f - fy) * top + fy * bot;
    }
    acc += row;
  }
  out[int64_t(plane) * opix + pix] = acc;
}

__global__ __launch_bounds__(256) void k_ref_ytab(GeomI g, const int32_t* __restrict__ itab,
                                                  const float* __restrict__ ftab, int64_t stride,
                                                  int first, int count, YEntry* __restrict__ ytab) {
  const int k = blockIdx.x;
  if (k >= count) return;
  const int plane = first + k;
  const int32_t* it = itab + int64_t(plane) * stride;
  const float* ft = ftab + int64_t(plane) * stride;
  const int e_by = g.out_w + g.out_h + g.wb;
  const int64_t n = int64_t(g.hb) * g.out_h;
  for (int64_t e = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; e < n;
       e += int64_t(gridDim.y) * blockDim.x) {
    const int yb = int(e / g.out_h), yr = int(e % g.out_h);
    int y0 = it[g.out_w + yr] + it[e_by + yb];
    float fy = ft[g.out_w + yr] + ft[e_by + yb];
    if (fy >= 1.0f) {
      y0 += 1;
      fy -= 1.0f;
    }
    YEntry v;
    clamp_cell(y0, fy, g.ha, v.row, v.w0, v.w1);
    v.pad = 0;
    ytab[int64_t(plane) * n + e] = v;
  }
}

// Window bounds of the batched kernel.  For plane group gq (planes
// gq*NW .. gq*NW+NW-1), tile column tx and lens-plane column x_b: the first and
// last interpolation column any sample of the group's planes can start in,
// clamped into [0, wa-2], the last one plus one for the right neighbour.
// Likewise for rows.  Integer parts at the tile's extreme columns / rows bound
// every sample because a_x and a_y are affine in the output coordinate.
__global__ __launch_bounds__(256) void k_ref_bounds(GeomI g, const int32_t* __restrict__ itab,
                                                    int64_t stride, int n_alpha, int nw, int rw,
                                                    int groups, int tiles_x, int tiles_y,
                                                    int2* __restrict__ bx, int2* __restrict__ by) {
  const int e_bx = g.out_w + g.out_h, e_by = e_bx + g.wb;
  const int64_t nxe = int64_t(groups) * tiles_x * g.wb;
  const int64_t nye = int64_t(groups) * tiles_y * g.hb;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < nxe + nye;
       e += int64_t(gridDim.x) * 256) {
    const bool is_x = e < nxe;
    const int64_t f = is_x ? e : e - nxe;
    const int nb = is_x ? g.wb : g.hb;
    const int nt = is_x ? tiles_x : tiles_y;
    const int vb = int(f % nb);
    const int t = int((f / nb) % nt);
    const int gq = int(f / (int64_t(nb) * nt));
    const int tsz = is_x ? 64 : rw;
    const int lim = is_x ? g.out_w : g.out_h;
    const int lo_o = t * tsz;
    const int hi_o = (lo_o + tsz - 1) < lim ? lo_o + tsz - 1 : lim - 1;
    const int ea = is_x ? 0 : g.out_w;
    const int eb = (is_x ? e_bx : e_by) + vb;
    int lo = 1 << 30, hi = -(1 << 30);
    for (int k = 0; k < nw; ++k) {
      const int pk = (gq * nw + k) < n_alpha ? gq * nw + k : n_alpha - 1;
      const int32_t* it = itab + int64_t(pk) * stride;
      const int a0 = it[ea + lo_o], a1 = it[ea + hi_o], ib = it[eb];
      lo = min(lo, min(a0, a1) + ib);
      hi = max(hi, max(a0, a1) + ib + 1);
    }
    const int size = is_x ? g.wa : g.ha;
    lo = min(max(lo, 0), size - 2);
    hi = min(max(hi, 0), size - 2) + 1;
    if (is_x)
      bx[f] = make_int2(lo, hi);
    else
      by[f] = make_int2(lo, hi);
  }
}

// Batched refocus.  A work-group of NW waves covers one output tile of 64
// columns x RW rows for NW consecutive planes (wave w = plane k0 + w) and one
// slice of view rows; lane = column.
//
// For every view the union of the NW planes' sample footprints over the tile
// is a small window of that view.  Windows are copied straight from global
// memory into LDS (global_load_lds, no registers), double-buffered: the copy
// of view v+1 is in flight while view v is interpolated, with one barrier per
// view.  Rows have a fixed stride of kWinStride floats, so the two taps of a
// row are adjacent and the next row is a constant offset away.  When view
// rows are a multiple of 4 floats long, the window starts on a 4-float
// boundary and each copy instruction moves two window rows, 16 bytes per
// lane; otherwise one float per lane.  A view whose window does not fit is
// read with direct paired gathers instead; both paths give identical results.
// Column coordinates are computed per lane for the wave's own plane and
// reused for its RW rows; row coordinates come from the row table as
// wave-uniform (scalar) values.
constexpr int kWinStride = 128;           // LDS row stride (floats) = max window width
constexpr int kWinRows = 64;              // max window height

typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

struct Window {
  int x0, y0, w, h;   // window origin and size in view pixels
  bool fits;
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

template <int NW, int RW>
__global__ __launch_bounds__(NW * 64) void k_ref_batched(
    const float* __restrict__ gamma, GeomI g, const int32_t* __restrict__ itab,
    const float* __restrict__ ftab, const YEntry* __restrict__ ytab,
    const int2* __restrict__ bx, const int2* __restrict__ by, int64_t stride, int n_alpha,
    int tiles_x, int tiles_y, int groups, int splits, int yb_per_split, float* __restrict__ dst,
    int64_t split_stride) {
  __shared__ float win0[kWinRows * kWinStride];
  __shared__ float win1[kWinRows * kWinStride];
  int b = blockIdx.x;
  const int split = b % splits;
  b /= splits;
  const int grp = b % groups;
  b /= groups;
  const int tile_x = b % tiles_x, tile_y = b / tiles_x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int xr = tile_x * 64 + lane;
  const int xrc = xr < g.out_w ? xr : g.out_w - 1;
  const int k0 = grp * NW;
  const int plane = (k0 + wave) < n_alpha ? k0 + wave : n_alpha - 1;
  const int64_t pa = int64_t(g.wa) * g.ha;
  const int e_bx = g.out_w + g.out_h, e_by = e_bx + g.wb;
  const int ty_lo = tile_y * RW;

  // column coordinates of this lane in this wave's plane
  const int32_t* itw = itab + int64_t(plane) * stride;
  const float* ftw = ftab + int64_t(plane) * stride;
  const int iax = itw[xrc];
  const float fax = ftw[xrc];
  const YEntry* yw = ytab + int64_t(plane) * g.hb * g.out_h;
  const int2* bxw = bx + (int64_t(grp) * tiles_x + tile_x) * g.wb;
  const int2* byw = by + (int64_t(grp) * tiles_y + tile_y) * g.hb;

  const bool quad = (g.wa & 3) == 0;
  auto window = [&](int yb, int xb) {
    const int2 cx = bxw[xb], cy = byw[yb];
    Window w;
    w.x0 = quad ? (cx.x & ~3) : cx.x;
    w.y0 = cy.x;
    w.w = cx.y - w.x0 + 1;
    if (quad) w.w = (w.w + 3) & ~3;   // stays within the view: wa is a multiple of 4
    w.h = cy.y - cy.x + 1;
    w.fits = w.w <= kWinStride && w.h <= kWinRows;
    return w;
  };
  // Copy a window into LDS.  16-byte copies: instruction i (waves take turns)
  // moves window rows 2i (lanes 0-31) and 2i+1 (lanes 32-63), 4 floats per
  // lane, which land in LDS exactly at those rows' kWinStride-float slots.
  // 4-byte copies: wave w copies rows w, w+NW, ...; lane l columns l and l+64.
  // Lanes beyond the window stay idle.
  auto copy_window = [&](const float* view, const Window& w, float* buf) {
    if (quad) {
      const int half = lane >> 5, c4 = (lane & 31) * 4;
      for (int i = wave; 2 * i < w.h; i += NW) {
        const int row = 2 * i + half;
        if (row < w.h && c4 < w.w)
          __builtin_amdgcn_global_load_lds(view + int64_t(w.y0 + row) * g.wa + w.x0 + c4,
                                           (lds_ptr_t)(buf + 2 * i * kWinStride), 16, 0, 0);
      }
      return;
    }
    for (int row = wave; row < w.h; row += NW) {
      const float* src = view + int64_t(w.y0 + row) * g.wa + w.x0;
      float* drow = buf + row * kWinStride;
      if (lane < w.w)
        __builtin_amdgcn_global_load_lds(src + lane, (lds_ptr_t)drow, 4, 0, 0);
      if (64 + lane < w.w)
        __builtin_amdgcn_global_load_lds(src + 64 + lane, (lds_ptr_t)(drow + 64), 4, 0, 0);
    }
  };

  float acc[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) acc[r] = 0.0f;

  const int yb0 = split * yb_per_split;
  const int yb1 = (yb0 + yb_per_split) < g.hb ? yb0 + yb_per_split : g.hb;
  const int nview = (yb1 - yb0) * g.wb;
  Window wn = window(yb0, 0);
  if (wn.fits) copy_window(gamma + int64_t(yb0) * g.wb * pa, wn, win0);

  for (int yb = yb0; yb < yb1; ++yb) {
    YEntry yq[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int yr = ty_lo + r < g.out_h ? ty_lo + r : g.out_h - 1;
      yq[r] = yw[int64_t(yb) * g.out_h + yr];
    }
    float racc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) racc[r] = 0.0f;
    const float* vrow = gamma + int64_t(yb) * g.wb * pa;
    for (int xb = 0; xb < g.wb; ++xb) {
      const Window wc = wn;
      const float* view = vrow + int64_t(xb) * pa;
      const int vi = (yb - yb0) * g.wb + xb;
      float* cur = (vi & 1) ? win1 : win0;
      float* nxt = (vi & 1) ? win0 : win1;
      // This view's copy is complete for every wave, and every wave is done
      // with the previous view, whose buffer the next copy reuses.
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
      __syncthreads();
      if (vi + 1 < nview) {
        const int nyb = yb0 + (vi + 1) / g.wb, nxb = (vi + 1) % g.wb;
        wn = window(nyb, nxb);
        if (wn.fits) copy_window(gamma + (int64_t(nyb) * g.wb + nxb) * pa, wn, nxt);
      }
      int x0 = iax + itw[e_bx + xb];
      float fx = fax + ftw[e_bx + xb];
      if (fx >= 1.0f) {
        x0 += 1;
        fx -= 1.0f;
      }
      int xc;
      float wx0, wx1;
      clamp_cell(x0, fx, g.wa, xc, wx0, wx1);
      if (wc.fits) {
        const float* wl = cur + (xc - wc.x0);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const float* p = wl + (yq[r].row - wc.y0) * kWinStride;
          const float g00 = p[0], g01 = p[1], g10 = p[kWinStride], g11 = p[kWinStride + 1];
          const float top = __builtin_fmaf(wx1, g01, wx0 * g00);
          const float bot = __builtin_fmaf(wx1, g11, wx0 * g10);
          racc[r] = __builtin_fmaf(yq[r].w0, top, racc[r]);
          racc[r] = __builtin_fmaf(yq[r].w1, bot, racc[r]);
        }
      } else {
        const float* vx = view + xc;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const float* p = vx + int64_t(yq[r].row) * g.wa;
          const f2u t0 = *reinterpret_cast<const f2u*>(p);
          const f2u t1 = *reinterpret_cast<const f2u*>(p + g.wa);
          const float top = __builtin_fmaf(wx1, t0.y, wx0 * t0.x);
          const float bot = __builtin_fmaf(wx1, t1.y, wx0 * t1.x);
          racc[r] = __builtin_fmaf(yq[r].w0, top, racc[r]);
          racc[r] = __builtin_fmaf(yq[r].w1, bot, racc[r]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] += racc[r];
  }

  const int64_t opix = int64_t(g.out_w) * g.out_h;
  float* d = dst + int64_t(split) * split_stride;
  if (xr < g.out_w && k0 + wave < n_alpha) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int yr = ty_lo + r;
      if (yr < g.out_h) d[int64_t(k0 + wave) * opix + int64_t(yr) * g.out_w + xr] = acc[r];
    }
  }
}

// Separable batched refocus.  The row side of a sample (clamped row c and
// weights w0, w1) depends on (plane, y_b, y_r) only, not on x_b, so for one
// lens-plane row y_b the column interpolation can be summed over x_b first:
//     H[y] = sum over x_b of (wx0 * view(y, xc) + wx1 * view(y, xc + 1)),
// one value per view row y that any of the tile's output rows touches, and
//     out(y_r) += w0 * H[c] + w1 * H[c + 1]
// once per y_b.  Per view and wave that is one column pair per touched row
// (about alpha * RW + 2 rows) instead of two pairs and the row weights per
// output row.  Work decomposition, window bounds and coordinate arithmetic
// are those of k_ref_batched.
//
// Windows are staged S views deep (S - 1 copies in flight while one is
// read).  Every wave issues the same number of copy instructions per view,
// so one vmcnt immediate separates the views; only lanes inside the window
// fetch.  Per-view bookkeeping touches no memory: the per-x_b values (the
// wave's column integer part and fraction, the window's first column and
// width) sit one per lane for 64 lens-plane columns at a time and are read
// with readlane; the row entries of the tile sit one per lane and are loaded
// once per y_b.  A lens-plane row whose windows do not fit, and every row of
// a group whose planes touch more view rows than the registers hold
// (|alpha| above about 2), is summed from direct paired gathers, as in
// k_ref_batched.

// Window rows per stage (the union over the group's planes, whose shifts
// differ): 2 RW, plus 32 for groups of 8 or more planes; a multiple of 2 NW.
constexpr int sep_window_rows(int nw, int rw) {
  return ((2 * rw + (nw >= 8 ? 32 : 0) + 2 * nw - 1) / (2 * nw)) * (2 * nw);
}

template <int NW, int RW>
struct SepShape {
  // view rows one plane's tile touches, held in registers: up to 2 RW
  // (|alpha| up to about 2)
  static constexpr int nh = 2 * RW;
  static constexpr int rows = sep_window_rows(NW, RW);
  static constexpr int cp16 = rows / (2 * NW);   // 16-byte copies per wave per view
  static constexpr int cp4 = 2 * rows / NW;      // 4-byte copies per wave per view
};

constexpr int kSepBlk = 8;   // rows per guarded block of the column sums

// LDS of k_ref_sep<NW, RW, S>: S window stages plus kSepBlk rows of padding.
template <int NW, int RW, int S>
constexpr int sep_lds_bytes() {
  return (S * SepShape<NW, RW>::rows + kSepBlk) * kWinStride * 4;
}
constexpr int kMaxLds = 160 * 1024;

typedef float f2 __attribute__((ext_vector_type(2)));

// Eight consecutive window rows (kWinStride floats apart) at LDS byte address
// a: c0[k] = rows 2k, 2k+1 at the lane's column, c1[k] = the next column.
// Inline asm with its own wait: the compiler would otherwise wait for every
// global->LDS copy in flight before each LDS read.
__device__ __forceinline__ void lds_rows8(uint32_t a, f2 (&c0)[4], f2 (&c1)[4]) {
  static_assert(kWinStride == 128, "offsets below are in units of 64 floats");
  asm volatile(
      "ds_read2st64_b32 %0, %8 offset1:2\n"
      "ds_read2st64_b32 %1, %8 offset0:4 offset1:6\n"
      "ds_read2st64_b32 %2, %8 offset0:8 offset1:10\n"
      "ds_read2st64_b32 %3, %8 offset0:12 offset1:14\n"
      "ds_read2st64_b32 %4, %9 offset1:2\n"
      "ds_read2st64_b32 %5, %9 offset0:4 offset1:6\n"
      "ds_read2st64_b32 %6, %9 offset0:8 offset1:10\n"
      "ds_read2st64_b32 %7, %9 offset0:12 offset1:14\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(c0[0]), "=&v"(c0[1]), "=&v"(c0[2]), "=&v"(c0[3]), "=&v"(c1[0]), "=&v"(c1[1]),
        "=&v"(c1[2]), "=&v"(c1[3])
      : "v"(a), "v"(a + 4u));
}

__device__ __forceinline__ int lane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

template <int NW, int RW, int S>
__global__ __launch_bounds__(NW * 64, 4) void k_ref_sep(
    const float* __restrict__ gamma, GeomI g, const int32_t* __restrict__ itab,
    const float* __restrict__ ftab, const YEntry* __restrict__ ytab,
    const int2* __restrict__ bx, const int2* __restrict__ by, int64_t stride, int n_alpha,
    int tiles_x, int tiles_y, int groups, int splits, int yb_per_split, float* __restrict__ dst,
    int64_t split_stride) {
  typedef SepShape<NW, RW> Sh;
  constexpr int WR = Sh::rows;
  constexpr int NH = Sh::nh;
  static_assert(NH % kSepBlk == 0 && kSepBlk == 8, "row blocks of lds_rows8");
  static_assert(RW <= 64, "row entries one per lane");
  // S window stages plus kSepBlk rows of padding: a row block may read up to
  // kSepBlk - 1 rows past a window (values never used).
  __shared__ float ring[(S * WR + kSepBlk) * kWinStride];
  int b = blockIdx.x;
  const int split = b % splits;
  b /= splits;
  const int grp = b % groups;
  b /= groups;
  const int tile_x = b % tiles_x, tile_y = b / tiles_x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int xr = tile_x * 64 + lane;
  const int xrc = xr < g.out_w ? xr : g.out_w - 1;
  const int k0 = grp * NW;
  const int plane = (k0 + wave) < n_alpha ? k0 + wave : n_alpha - 1;
  const int64_t pa = int64_t(g.wa) * g.ha;
  const int wb = g.wb;
  const int e_bx = g.out_w + g.out_h;
  const int ty_lo = tile_y * RW;

  const int32_t* itw = itab + int64_t(plane) * stride;
  const float* ftw = ftab + int64_t(plane) * stride;
  const int iax = itw[xrc];
  const float fax = ftw[xrc];
  const YEntry* yw = ytab + int64_t(plane) * g.hb * g.out_h;
  const int2* bxw = bx + (int64_t(grp) * tiles_x + tile_x) * wb;
  const int2* byw = by + (int64_t(grp) * tiles_y + tile_y) * g.hb;
  const bool quad = (g.wa & 3) == 0;

  // Column window of lens-plane column xb: first column (a multiple of 4 for
  // 16-byte copies) and width.
  auto xwin = [&](int xb, int& x0, int& w) {
    const int2 cx = bxw[xb];
    x0 = quad ? (cx.x & ~3) : cx.x;
    w = cx.y - x0 + 1;
    if (quad) w = (w + 3) & ~3;   // stays within the view: wa is a multiple of 4
  };
  // Whether every column window fits (they depend on x_b only).
  bool xfit = true;
  for (int c0 = 0; c0 < wb; c0 += 64) {
    int x0 = 0, w = 0;
    if (c0 + lane < wb) xwin(c0 + lane, x0, w);
    xfit = xfit && __builtin_amdgcn_ballot_w64(w > kWinStride) == 0;
  }

  // Rows one plane's tile touches at any y_b: the clamped rows
  // iay(y_r) + iby(y_b) + carry span at most |iay(last) - iay(first)| + 1
  // (iay is monotone in y_r), plus the cell's second row.  The largest span
  // over the group's planes decides (for the whole work-group) whether the
  // register rows suffice.
  int span = 0;
  {
    const int y_last = ty_lo + RW - 1 < g.out_h ? ty_lo + RW - 1 : g.out_h - 1;
    for (int k = 0; k < NW; ++k) {
      const int pk = (k0 + k) < n_alpha ? k0 + k : n_alpha - 1;
      const int32_t* it = itab + int64_t(pk) * stride + g.out_w;
      const int d = it[y_last] - it[ty_lo];
      span = max(span, (d < 0 ? -d : d) + 3);
    }
  }
  const bool rows_fit = span <= NH;

  const int yb0 = split * yb_per_split;
  const int yb1 = (yb0 + yb_per_split) < g.hb ? yb0 + yb_per_split : g.hb;
  const int nview = (yb1 - yb0) * wb;

  // ---- copy side: view iss_v (running index over this split's views) at
  // lens-plane (iss_yb, iss_xb); per-lane column windows of chunk iss_chunk.
  int iss_v = 0, iss_yb = yb0, iss_xb = 0, iss_stage = 0;
  int iss_chunk = -1, iss_cx0 = 0, iss_cw = 0;
  int2 iss_cy = byw[yb0];
  // Copy view iss_v into stage iss_v % S: its window, or an in-bounds
  // placeholder when it is past the last view or its window does not fit.
  // Every wave issues Sh::cp16 (16-byte) or Sh::cp4 (4-byte) instructions;
  // only lanes inside the window fetch, except lane 0, which always copies
  // (a clamped, in-bounds address into an LDS slot no sample reads) so that
  // no instruction is skipped for an empty exec mask.
  auto issue_next = [&]() {
    Window w;
    const float* view = gamma;
    bool real = false;
    if (iss_v < nview) {
      const int c = iss_xb >> 6;
      if (c != iss_chunk) {
        iss_cx0 = 0;
        iss_cw = 0;
        if (iss_xb - (iss_xb & 63) + lane < wb) xwin(iss_xb - (iss_xb & 63) + lane, iss_cx0, iss_cw);
        iss_chunk = c;
      }
      w.x0 = lane_i(iss_cx0, iss_xb & 63);
      w.w = lane_i(iss_cw, iss_xb & 63);
      w.y0 = iss_cy.x;
      w.h = iss_cy.y - iss_cy.x + 1;
      real = xfit && rows_fit && w.w <= kWinStride && w.h <= WR;
      view = gamma + (int64_t(iss_yb) * wb + iss_xb) * pa;
    }
    if (!real) {
      w.x0 = 0;
      w.y0 = 0;
      w.w = g.wa < 4 ? g.wa : 4;   // (a multiple of 4 when the rows are)
      w.h = 1;
    }
    float* buf = ring + iss_stage * (WR * kWinStride);
    if (quad) {
      const int half = lane >> 5;
      const int c4 = (lane & 31) * 4;
#pragma unroll
      for (int j = 0; j < Sh::cp16; ++j) {
        const int i = wave + j * NW;   // window row pair
        const int row = 2 * i + half;
        if ((row < w.h && c4 < w.w) || lane == 0) {
          const int srow = row < w.h ? row : w.h - 1;
          __builtin_amdgcn_global_load_lds(view + int64_t(w.y0 + srow) * g.wa + w.x0 + c4,
                                           (lds_ptr_t)(buf + 2 * i * kWinStride), 16, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < Sh::cp4 / 2; ++j) {
        const int row = wave + j * NW;
        const int srow = row < w.h ? row : w.h - 1;
        const float* src = view + int64_t(w.y0 + srow) * g.wa + w.x0;
        if ((row < w.h && lane < w.w) || lane == 0)
          __builtin_amdgcn_global_load_lds(src + lane, (lds_ptr_t)(buf + row * kWinStride), 4, 0,
                                           0);
        if ((row < w.h && 64 + lane < w.w) || lane == 0) {
          const int c1 = 64 < w.w ? 64 + lane : w.w - 1;
          __builtin_amdgcn_global_load_lds(src + c1, (lds_ptr_t)(buf + row * kWinStride + 64), 4,
                                           0, 0);
        }
      }
    }
    ++iss_v;
    iss_stage = iss_stage + 1 == S ? 0 : iss_stage + 1;
    if (++iss_xb == wb) {
      iss_xb = 0;
      ++iss_yb;
      if (iss_yb < yb1) iss_cy = byw[iss_yb];
    }
  };
  // Every view starts with: this wave's copies of view vi are complete (the
  // S - 2 later views' copies may still be in flight), then a bare barrier
  // makes them complete for every wave and guarantees every wave is done with
  // view vi - 1, whose stage the next copy reuses.  (__syncthreads() would
  // also wait for every copy in flight; this wave's LDS reads of view vi - 1
  // have completed, each read group waits for itself.)
  // The counter holds at most 63: where the copies of S - 1 views could
  // exceed that, wait for all of them instead.
  constexpr int kAhead16 = (S - 1) * Sh::cp16 <= 63 ? (S - 2) * Sh::cp16 : 0;
  constexpr int kAhead4 = (S - 1) * Sh::cp4 <= 63 ? (S - 2) * Sh::cp4 : 0;
  auto next_view = [&]() {
    if (quad)
      wait_vmcnt<kAhead16>();
    else
      wait_vmcnt<kAhead4>();
    __builtin_amdgcn_s_barrier();
    issue_next();
  };

  // ---- compute side: per-lane values of chunk col_chunk for this wave's
  // plane: column integer part and fraction, window first column.
  int col_chunk = -1, col_i = 0, col_x0 = 0;
  float col_f = 0.0f;
  auto column = [&](int xb, int& xc, float& wx0, float& wx1, int& wx) {
    const int c = xb >> 6;
    if (c != col_chunk) {
      const int xl = xb - (xb & 63) + lane;
      col_i = 0;
      col_f = 0.0f;
      col_x0 = 0;
      if (xl < wb) {
        col_i = itw[e_bx + xl];
        col_f = ftw[e_bx + xl];
        int w;
        xwin(xl, col_x0, w);
      }
      col_chunk = c;
    }
    int x0 = iax + lane_i(col_i, xb & 63);
    float fx = fax + lane_f(col_f, xb & 63);
    if (fx >= 1.0f) {
      x0 += 1;
      fx -= 1.0f;
    }
    clamp_cell(x0, fx, g.wa, xc, wx0, wx1);
    wx = lane_i(col_x0, xb & 63);
  };

  float acc[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) acc[r] = 0.0f;

#pragma unroll
  for (int v = 0; v < S - 1; ++v) issue_next();

  int stage = 0;   // stage of view vi
  for (int yb = yb0; yb < yb1; ++yb) {
    // row entries of the tile's output rows, one per lane (lane r: row r)
    int yrow = 0;
    float yw0 = 0.0f, yw1 = 0.0f;
    if (lane < RW) {
      const int yr = ty_lo + lane < g.out_h ? ty_lo + lane : g.out_h - 1;
      const YEntry e = yw[int64_t(yb) * g.out_h + yr];
      yrow = e.row;
      yw0 = e.w0;
      yw1 = e.w1;
    }
    int ylo = 1 << 30, yhi = -(1 << 30);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = lane_i(yrow, r);
      ylo = min(ylo, row);
      yhi = max(yhi, row + 1);
    }
    const int nh = yhi - ylo + 1;
    const int2 cy = byw[yb];
    const bool sep = xfit && rows_fit && (cy.y - cy.x + 1) <= WR;
    if (sep) {
      float H[NH];
#pragma unroll
      for (int i = 0; i < NH; ++i) H[i] = 0.0f;
      const uint32_t rbase =
          uint32_t(reinterpret_cast<uintptr_t>(ring)) + uint32_t((ylo - cy.x) * kWinStride * 4);
      for (int xb = 0; xb < wb; ++xb) {
        next_view();
        int xc, wxs;
        float wx0, wx1;
        column(xb, xc, wx0, wx1, wxs);
        const uint32_t a0 =
            rbase + uint32_t(stage * (WR * kWinStride * 4)) + uint32_t((xc - wxs) * 4);
        stage = stage + 1 == S ? 0 : stage + 1;
#pragma unroll
        for (int blk = 0; blk < NH / kSepBlk; ++blk) {
          if (blk * kSepBlk < nh) {
            f2 c0[4], c1[4];
            lds_rows8(a0 + blk * kSepBlk * kWinStride * 4, c0, c1);
#pragma unroll
            for (int t = 0; t < kSepBlk; ++t) {
              const int i = blk * kSepBlk + t;
              const float g0 = c0[t >> 1][t & 1], g1 = c1[t >> 1][t & 1];
              H[i] = __builtin_fmaf(wx0, g0, H[i]);
              H[i] = __builtin_fmaf(wx1, g1, H[i]);
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int i0 = lane_i(yrow, r) - ylo;   // wave-uniform, i0 + 1 < nh
        acc[r] += __builtin_fmaf(lane_f(yw1, r), H[i0 + 1], lane_f(yw0, r) * H[i0]);
      }
    } else {
      float racc[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) racc[r] = 0.0f;
      const float* vrow = gamma + int64_t(yb) * wb * pa;
      for (int xb = 0; xb < wb; ++xb) {
        next_view();
        stage = stage + 1 == S ? 0 : stage + 1;
        int xc, wxs;
        float wx0, wx1;
        column(xb, xc, wx0, wx1, wxs);
        const float* vx = vrow + int64_t(xb) * pa + xc;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const float* p = vx + int64_t(lane_i(yrow, r)) * g.wa;
          const f2u t0 = *reinterpret_cast<const f2u*>(p);
          const f2u t1 = *reinterpret_cast<const f2u*>(p + g.wa);
          const float top = __builtin_fmaf(wx1, t0.y, wx0 * t0.x);
          const float bot = __builtin_fmaf(wx1, t1.y, wx0 * t1.x);
          racc[r] = __builtin_fmaf(lane_f(yw0, r), top, racc[r]);
          racc[r] = __builtin_fmaf(lane_f(yw1, r), bot, racc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < RW; ++r) acc[r] += racc[r];
    }
  }
  // Drain the placeholder copies issued past the last view.
  wait_vmcnt<0>();

  const int64_t opix = int64_t(g.out_w) * g.out_h;
  float* d = dst + int64_t(split) * split_stride;
  if (xr < g.out_w && k0 + wave < n_alpha) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int yr = ty_lo + r;
      if (yr < g.out_h) d[int64_t(k0 + wave) * opix + int64_t(yr) * g.out_w + xr] = acc[r];
    }
  }
}

// out[i] = sum over s of partial[s*stride + i], in order s = 0, 1, ...
__global__ __launch_bounds__(256) void k_sum_splits(const float* __restrict__ partial,
                                                    int splits, int64_t stride, int64_t count,
                                                    float* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * 256) {
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += partial[int64_t(k) * stride + i];
    out[i] = s;
  }
}

template <int NW, int RW, int MODE>
hipError_t launch_batched(const float* gamma, const GeomI& gi, const int32_t* itab,
                          const float* ftab, const YEntry* ytab, int2* bounds, int64_t stride,
                          int n_alpha, int splits, float* partial, float* out, hipStream_t s) {
  const int tiles_x = (gi.out_w + 63) / 64;
  const int tiles_y = (gi.out_h + RW - 1) / RW;
  const int groups = (n_alpha + NW - 1) / NW;
  if (splits > gi.hb) splits = gi.hb;
  if (splits < 1) splits = 1;
  const int ybs = (gi.hb + splits - 1) / splits;
  splits = (gi.hb + ybs - 1) / ybs;
  const int64_t nwg = int64_t(tiles_x) * tiles_y * groups * splits;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t opix = int64_t(gi.out_w) * gi.out_h;
  const int64_t count = opix * n_alpha;
  float* dst = splits > 1 ? partial : out;
  int2* bx = bounds;
  int2* by = bounds + int64_t(groups) * tiles_x * gi.wb;
  const int64_t nb = int64_t(groups) * (int64_t(tiles_x) * gi.wb + int64_t(tiles_y) * gi.hb);
  int64_t gb = (nb + 255) / 256;
  if (gb > 4096) gb = 4096;
  hipLaunchKernelGGL(k_ref_bounds, dim3(unsigned(gb)), dim3(256), 0, s, gi, itab, stride, n_alpha,
                     NW, RW, groups, tiles_x, tiles_y, bx, by);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr (MODE == 0)
    hipLaunchKernelGGL((k_ref_batched<NW, RW>), dim3(unsigned(nwg)), dim3(NW * 64), 0, s, gamma,
                       gi, itab, ftab, ytab, bx, by, stride, n_alpha, tiles_x, tiles_y, groups,
                       splits, ybs, dst, count);
  else if constexpr (sep_lds_bytes<NW, RW, MODE>() <= kMaxLds)
    hipLaunchKernelGGL((k_ref_sep<NW, RW, MODE>), dim3(unsigned(nwg)), dim3(NW * 64), 0, s,
                       gamma, gi, itab, ftab, ytab, bx, by, stride, n_alpha, tiles_x, tiles_y,
                       groups, splits, ybs, dst, count);
  else
    return hipErrorInvalidValue;
  e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  int64_t gr = (count + 255) / 256;
  if (gr > 16384) gr = 16384;
  hipLaunchKernelGGL(k_sum_splits, dim3(unsigned(gr)), dim3(256), 0, s, partial, splits, count,
                     count, out);
  return hipGetLastError();
}

// Views of Gamma resampled along the lens-plane coordinate: output view
// s = j * nx + i is the bilinear interpolant of the views at the sample point
// (x_b, y_b) = (ox + i sx, oy + j sy), i.e. the sum over its four neighbouring
// views (x_b0 + ex, y_b0 + ey) weighted by (1 - f or f) products, views outside
// detector B contributing zero.  Sample parameters are FP64, weights FP32.
// One work-group row per sample (grid-stride over samples), 4 values per
// thread when pa % 4 == 0.
__global__ __launch_bounds__(256) void k_resample_views(const float* __restrict__ gamma,
                                                        int64_t pa, int wb, int hb, int nx,
                                                        int ny, double ox, double oy, double sx,
                                                        double sy, float* __restrict__ out) {
  const int64_t ns = int64_t(nx) * ny;
  for (int64_t s = blockIdx.y; s < ns; s += gridDim.y) {
    const int i = int(s % nx), j = int(s / nx);
    const double xb = ox + double(i) * sx, yb = oy + double(j) * sy;
    const double fxb = floor(xb), fyb = floor(yb);
    const int x0 = int(fxb), y0 = int(fyb);
    const double fx = xb - fxb, fy = yb - fyb;
    const float* src[4];
    float w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int ex = c & 1, ey = c >> 1;
      const int cx = x0 + ex, cy = y0 + ey;
      const double wd = (ey ? fy : 1.0 - fy) * (ex ? fx : 1.0 - fx);
      const bool in = cx >= 0 && cx < wb && cy >= 0 && cy < hb && wd != 0.0;
      w[c] = in ? float(wd) : 0.0f;
      src[c] = in ? gamma + (int64_t(cy) * wb + cx) * pa : nullptr;
    }
    float* dst = out + s * pa;
    if ((pa & 3) == 0) {
      const int64_t n4 = pa >> 2;
      for (int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x; q < n4;
           q += int64_t(gridDim.x) * 256) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (!src[c]) continue;
          const float4 v = reinterpret_cast<const float4*>(src[c])[q];
          acc.x = fmaf(w[c], v.x, acc.x);
          acc.y = fmaf(w[c], v.y, acc.y);
          acc.z = fmaf(w[c], v.z, acc.z);
          acc.w = fmaf(w[c], v.w, acc.w);
        }
        reinterpret_cast<float4*>(dst)[q] = acc;
      }
    } else {
      for (int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x; q < pa;
           q += int64_t(gridDim.x) * 256) {
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (src[c]) acc = fmaf(w[c], src[c][q], acc);
        dst[q] = acc;
      }
    }
  }
}

}  // namespace

hipError_t refocus_tables(const RefGeom& g, const double* alphas, int first, int count,
                          int64_t stride, int32_t* itab, float* ftab, void* ytab, hipStream_t s) {
  if (count < 1 || count > kAlphaPerLaunch) return hipErrorInvalidValue;
  AlphaPack ap;
  for (int k = 0; k < kAlphaPerLaunch; ++k) ap.a[k] = k < count ? alphas[first + k] : 0.0;
  hipLaunchKernelGGL(k_ref_tables, dim3(unsigned(count)), dim3(256), 0, s, ap, count, first, g,
                     stride, itab, ftab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !ytab) return e;
  const GeomI gi{g.wa, g.ha, g.wb, g.hb, g.out_w, g.out_h};
  int64_t gy = (int64_t(g.hb) * g.out_h + 255) / 256;   // entries per plane / 256
  if (gy > 64) gy = 64;
  hipLaunchKernelGGL(k_ref_ytab, dim3(unsigned(count), unsigned(gy)), dim3(256), 0, s, gi, itab,
                     ftab, stride, first, count, static_cast<YEntry*>(ytab));
  return hipGetLastError();
}

hipError_t refocus_plain(const float* gamma, const RefGeom& g, const int32_t* itab,
                         const float* ftab, int64_t stride, int plane, float* out,
                         hipStream_t s) {
  const GeomI gi{g.wa, g.ha, g.wb, g.hb, g.out_w, g.out_h};
  const int64_t opix = int64_t(g.out_w) * g.out_h;
  hipLaunchKernelGGL(k_ref_plain, dim3(unsigned((opix + 255) / 256)), dim3(256), 0, s, gamma, gi,
                     itab, ftab, stride, plane, out);
  return hipGetLastError();
}

bool refocus_config_supported(const RefocusConfig& c) {
  const bool pair_ok = (c.kp == 4 && (c.rw == 8 || c.rw == 16)) ||
                       (c.kp == 8 && (c.rw == 8 || c.rw == 16 || c.rw == 32)) ||
                       (c.kp == 16 && (c.rw == 8 || c.rw == 16));
  // column-sum kernel only: fewer planes per work-group, taller tiles
  const bool sep_pair = (c.kp == 1 && c.rw == 16) || (c.kp == 2 && (c.rw == 16 || c.rw == 32)) ||
                        (c.kp == 4 && c.rw == 32);
  if (c.mode == 2) return rows_config_built(c.kp, c.rw);
  const bool ok = c.mode == 0 ? pair_ok
                              : (c.mode == 1 && c.stages >= 2 && c.stages <= 4 &&
                                 (pair_ok || sep_pair));
  // the window stages of the column-sum kernel must fit in LDS
  const bool lds_ok =
      c.mode != 1 ||
      (c.kp > 0 && (c.stages * sep_window_rows(c.kp, c.rw) + kSepBlk) * kWinStride * 4 <= kMaxLds);
  return ok && lds_ok && c.splits >= 1 && c.splits <= kMaxViewSplits;
}

hipError_t refocus_batched(const float* gamma, const RefGeom& g, const int32_t* itab,
                           const float* ftab, const void* ytab, void* bounds, int64_t stride,
                           int n_alpha, const RefocusConfig& c, float* partial, float* out,
                           hipStream_t s) {
  const GeomI gi{g.wa, g.ha, g.wb, g.hb, g.out_w, g.out_h};
  const YEntry* yt = static_cast<const YEntry*>(ytab);
  int2* bd = static_cast<int2*>(bounds);
// MODE 0: k_ref_batched; MODE 2..4: k_ref_sep with that many copy stages.
#define CPI_REF_CASE(NW_, RW_)                                                             \
  if (c.kp == NW_ && c.rw == RW_) {                                                        \
    const int m = c.mode == 0 ? 0 : c.stages;                                              \
    if (m == 0)                                                                            \
      return launch_batched<NW_, RW_, 0>(gamma, gi, itab, ftab, yt, bd, stride, n_alpha,   \
                                         c.splits, partial, out, s);                       \
    if (m == 2)                                                                            \
      return launch_batched<NW_, RW_, 2>(gamma, gi, itab, ftab, yt, bd, stride, n_alpha,   \
                                         c.splits, partial, out, s);                       \
    if (m == 3)                                                                            \
      return launch_batched<NW_, RW_, 3>(gamma, gi, itab, ftab, yt, bd, stride, n_alpha,   \
                                         c.splits, partial, out, s);                       \
    if (m == 4)                                                                            \
      return launch_batched<NW_, RW_, 4>(gamma, gi, itab, ftab, yt, bd, stride, n_alpha,   \
                                         c.splits, partial, out, s);                       \
  }
// column-sum kernel only
#define CPI_REF_SEP_CASE(NW_, RW_)                                                         \
  if (c.kp == NW_ && c.rw == RW_ && c.mode == 1) {                                         \
    if (c.stages == 2)                                                                     \
      return launch_batched<NW_, RW_, 2>(gamma, gi, itab, ftab, yt, bd, stride, n_alpha,   \
                                         c.splits, partial, out, s);                       \
    if (c.stages == 3)                                                                     \
      return launch_batched<NW_, RW_, 3>(gamma, gi, itab, ftab, yt, bd, stride, n_alpha,   \
                                         c.splits, partial, out, s);                       \
    if (c.stages == 4)                                                                     \
      return launch_batched<NW_, RW_, 4>(gamma, gi, itab, ftab, yt, bd, stride, n_alpha,   \
                                         c.splits, partial, out, s);                       \
  }
  CPI_REF_SEP_CASE(1, 16)
  CPI_REF_SEP_CASE(2, 16)
  CPI_REF_SEP_CASE(2, 32)
  CPI_REF_SEP_CASE(4, 32)
  CPI_REF_CASE(4, 8)
  CPI_REF_CASE(4, 16)
  CPI_REF_CASE(8, 8)
  CPI_REF_CASE(8, 16)
  CPI_REF_CASE(8, 32)
  CPI_REF_CASE(16, 8)
  CPI_REF_CASE(16, 16)
#undef CPI_REF_CASE
#undef CPI_REF_SEP_CASE
  return hipErrorInvalidValue;
}

hipError_t resample_views(const float* gamma, int64_t pa, int wb, int hb, int nx, int ny, double ox,
                          double oy, double sx, double sy, float* out, hipStream_t s) {
  const int64_t ns = int64_t(nx) * ny;
  int64_t gx = (((pa & 3) == 0 ? pa / 4 : pa) + 255) / 256;
  if (gx > 64) gx = 64;
  const int64_t gy = ns < 65535 ? ns : 65535;
  hipLaunchKernelGGL(k_resample_views, dim3(unsigned(gx), unsigned(gy)), dim3(256), 0, s, gamma, pa,
                     wb, hb, nx, ny, ox, oy, sx, sy, out);
  return hipGetLastError();
}

}  // namespace cpi
