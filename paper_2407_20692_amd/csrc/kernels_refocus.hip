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
// row sums are summed over y_b (and, for the batched kernel, over view-row
// splits in a fixed order), so the result is bitwise reproducible for a
// given configuration.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpi {

namespace {

struct AlphaPack {
  double a[kAlphaPerLaunch];
};

struct GeomI {
  int wa, ha, wb, hb, out_w, out_h;
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

// Clamp an interpolation cell [i, i+1] into [0, size-2] and move the
// weights with it, zeroing taps that fall outside [0, size-1].  On return
// the two loaded taps are at c and c+1 with weights w0 and w1.
__device__ __forceinline__ void clamp_cell(int i, float f, int size, int& c, float& w0,
                                           float& w1) {
  const float a0 = (i >= 0 && i <= size - 1) ? 1.0f - f : 0.0f;   // tap i
  const float a1 = (i >= -1 && i <= size - 2) ? f : 0.0f;         // tap i + 1
  c = i < 0 ? 0 : (i > size - 2 ? size - 2 : i);
  w0 = (i == c) ? a0 : ((i == c - 1) ? a1 : 0.0f);
  w1 = (i == c) ? a1 : ((i == c + 1) ? a0 : 0.0f);
}

// Batched refocus: a work-group covers 64 output columns x (4*RW) rows for
// KP planes and one slice of view rows; lane = column, each wave RW rows.
template <int KP, int RW>
__global__ __launch_bounds__(256) void k_ref_batched(
    const float* __restrict__ gamma, GeomI g, const int32_t* __restrict__ itab,
    const float* __restrict__ ftab, int64_t stride, int n_alpha, int tiles_x, int groups,
    int splits, int yb_per_split, float* __restrict__ dst, int64_t split_stride) {
  int b = blockIdx.x;
  const int split = b % splits;
  b /= splits;
  const int grp = b % groups;
  b /= groups;
  const int tile_x = b % tiles_x, tile_y = b / tiles_x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int xr = tile_x * 64 + lane;
  const int xrc = xr < g.out_w ? xr : g.out_w - 1;
  const int yr0 = tile_y * (4 * RW) + wave * RW;
  const int k0 = grp * KP;
  const int64_t pa = int64_t(g.wa) * g.ha;
  const int e_bx = g.out_w + g.out_h, e_by = e_bx + g.wb;

  int iax[KP];
  float fax[KP];
  int iay[KP][RW];
  float fay[KP][RW];
  const int32_t* itk[KP];
  const float* ftk[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int plane = (k0 + k) < n_alpha ? k0 + k : n_alpha - 1;
    itk[k] = itab + int64_t(plane) * stride;
    ftk[k] = ftab + int64_t(plane) * stride;
    iax[k] = itk[k][xrc];
    fax[k] = ftk[k][xrc];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int yr = yr0 + r < g.out_h ? yr0 + r : g.out_h - 1;
      iay[k][r] = itk[k][g.out_w + yr];
      fay[k][r] = ftk[k][g.out_w + yr];
    }
  }

  float acc[KP][RW];
#pragma unroll
  for (int k = 0; k < KP; ++k)
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[k][r] = 0.0f;

  const int yb0 = split * yb_per_split;
  const int yb1 = (yb0 + yb_per_split) < g.hb ? yb0 + yb_per_split : g.hb;
  for (int yb = yb0; yb < yb1; ++yb) {
    int yoff[KP][RW];
    float wy0[KP][RW], wy1[KP][RW];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int iby = itk[k][e_by + yb];
      const float fby = ftk[k][e_by + yb];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        int y0 = iay[k][r] + iby;
        float fy = fay[k][r] + fby;
        if (fy >= 1.0f) {
          y0 += 1;
          fy -= 1.0f;
        }
        int c;
        clamp_cell(y0, fy, g.ha, c, wy0[k][r], wy1[k][r]);
        yoff[k][r] = c * g.wa;
      }
    }
    float racc[KP][RW];
#pragma unroll
    for (int k = 0; k < KP; ++k)
#pragma unroll
      for (int r = 0; r < RW; ++r) racc[k][r] = 0.0f;
    const float* vrow = gamma + int64_t(yb) * g.wb * pa;
    for (int xb = 0; xb < g.wb; ++xb) {
      const float* view = vrow + int64_t(xb) * pa;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        int x0 = iax[k] + itk[k][e_bx + xb];
        float fx = fax[k] + ftk[k][e_bx + xb];
        if (fx >= 1.0f) {
          x0 += 1;
          fx -= 1.0f;
        }
        int xc;
        float wx0, wx1;
        clamp_cell(x0, fx, g.wa, xc, wx0, wx1);
        const float* vx = view + xc;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const float* p = vx + yoff[k][r];
          const float g00 = p[0], g01 = p[1], g10 = p[g.wa], g11 = p[g.wa + 1];
          const float top = __builtin_fmaf(wx1, g01, wx0 * g00);
          const float bot = __builtin_fmaf(wx1, g11, wx0 * g10);
          racc[k][r] = __builtin_fmaf(wy0[k][r], top, racc[k][r]);
          racc[k][r] = __builtin_fmaf(wy1[k][r], bot, racc[k][r]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KP; ++k)
#pragma unroll
      for (int r = 0; r < RW; ++r) acc[k][r] += racc[k][r];
  }

  const int64_t opix = int64_t(g.out_w) * g.out_h;
  float* d = dst + int64_t(split) * split_stride;
  if (xr < g.out_w) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (k0 + k >= n_alpha) break;
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int yr = yr0 + r;
        if (yr < g.out_h) d[int64_t(k0 + k) * opix + int64_t(yr) * g.out_w + xr] = acc[k][r];
      }
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

template <int KP, int RW>
hipError_t launch_batched(const float* gamma, const GeomI& gi, const int32_t* itab,
                          const float* ftab, int64_t stride, int n_alpha, int splits,
                          float* partial, float* out, hipStream_t s) {
  const int tiles_x = (gi.out_w + 63) / 64;
  const int tiles_y = (gi.out_h + 4 * RW - 1) / (4 * RW);
  const int groups = (n_alpha + KP - 1) / KP;
  if (splits > gi.hb) splits = gi.hb;
  if (splits < 1) splits = 1;
  const int ybs = (gi.hb + splits - 1) / splits;
  splits = (gi.hb + ybs - 1) / ybs;
  const int64_t nwg = int64_t(tiles_x) * tiles_y * groups * splits;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t opix = int64_t(gi.out_w) * gi.out_h;
  const int64_t count = opix * n_alpha;
  float* dst = splits > 1 ? partial : out;
  hipLaunchKernelGGL((k_ref_batched<KP, RW>), dim3(unsigned(nwg)), dim3(256), 0, s, gamma, gi,
                     itab, ftab, stride, n_alpha, tiles_x, groups, splits, ybs, dst, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  int64_t gr = (count + 255) / 256;
  if (gr > 16384) gr = 16384;
  hipLaunchKernelGGL(k_sum_splits, dim3(unsigned(gr)), dim3(256), 0, s, partial, splits, count,
                     count, out);
  return hipGetLastError();
}

}  // namespace

hipError_t refocus_tables(const RefGeom& g, const double* alphas, int first, int count,
                          int64_t stride, int32_t* itab, float* ftab, hipStream_t s) {
  if (count < 1 || count > kAlphaPerLaunch) return hipErrorInvalidValue;
  AlphaPack ap;
  for (int k = 0; k < kAlphaPerLaunch; ++k) ap.a[k] = k < count ? alphas[first + k] : 0.0;
  hipLaunchKernelGGL(k_ref_tables, dim3(unsigned(count)), dim3(256), 0, s, ap, count, first, g,
                     stride, itab, ftab);
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
  const bool kp_ok = c.kp == 1 || c.kp == 2 || c.kp == 4 || c.kp == 8;
  const bool rw_ok = c.rw == 1 || c.rw == 2 || c.rw == 4 || c.rw == 8;
  return kp_ok && rw_ok && c.kp * c.rw <= 32 && c.splits >= 1 && c.splits <= kMaxViewSplits;
}

hipError_t refocus_batched(const float* gamma, const RefGeom& g, const int32_t* itab,
                           const float* ftab, int64_t stride, int n_alpha,
                           const RefocusConfig& c, float* partial, float* out,
                           hipStream_t s) {
  const GeomI gi{g.wa, g.ha, g.wb, g.hb, g.out_w, g.out_h};
#define CPI_REF_CASE(KP_, RW_)                                                               \
  if (c.kp == KP_ && c.rw == RW_)                                                            \
    return launch_batched<KP_, RW_>(gamma, gi, itab, ftab, stride, n_alpha, c.splits, partial, \
                                    out, s);
  CPI_REF_CASE(1, 1)
  CPI_REF_CASE(1, 2)
  CPI_REF_CASE(1, 4)
  CPI_REF_CASE(1, 8)
  CPI_REF_CASE(2, 1)
  CPI_REF_CASE(2, 2)
  CPI_REF_CASE(2, 4)
  CPI_REF_CASE(2, 8)
  CPI_REF_CASE(4, 1)
  CPI_REF_CASE(4, 2)
  CPI_REF_CASE(4, 4)
  CPI_REF_CASE(4, 8)
  CPI_REF_CASE(8, 1)
  CPI_REF_CASE(8, 2)
  CPI_REF_CASE(8, 4)
#undef CPI_REF_CASE
  return hipErrorInvalidValue;
}

}  // namespace cpi
