// Plain FP32 correlator: the comparison path for the int8 matrix-core one.
//
// Frames are unpacked to FP32 frame-major matrices (the paper's prototype
// also unpacks before multiplying, Section 4.1), per-pixel sums are FP32, and
// S_ab is an FP32 FMA matrix product on the vector ALUs (LDS-tiled, 8 x 8
// outputs per thread).  Gamma follows Eq. (1) term by term in FP32:
//     gamma_f32 = fl(S_ab / N) - fl(fl(S_a / N) * fl(S_b / N)).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpi {

namespace {

// out[f][p] = value of pixel p in frame f (0 for f >= n or p >= npix);
// colsum[p] += that value over the thread's frame slice.
__global__ __launch_bounds__(256) void k_unpack_f32(const uint8_t* __restrict__ frames, int fmt,
                                                    int64_t n, int64_t npix, int64_t kpad,
                                                    int64_t cols_pad, int64_t frames_per_slice,
                                                    float* __restrict__ out,
                                                    float* __restrict__ colsum) {
  const int64_t c0 = (int64_t(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (c0 >= cols_pad) return;
  const int64_t f0 = int64_t(blockIdx.y) * frames_per_slice;
  int64_t f1 = f0 + frames_per_slice;
  if (f1 > kpad) f1 = kpad;
  const int64_t fb = (fmt == CPI_FRAMES_U8) ? npix : (npix + 7) / 8;
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t f = f0; f < f1; ++f) {
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (f < n) {
      const uint8_t* row = frames + f * fb;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t p = c0 + b;
        if (p < npix) {
          uint32_t x;
          if (fmt == CPI_FRAMES_U8)
            x = row[p];
          else
            x = (uint32_t(row[p >> 3]) >> (p & 7)) & 1u;
          v[b] = float(x);
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) s[b] += v[b];
    *reinterpret_cast<float4*>(out + f * cols_pad + c0) = make_float4(v[0], v[1], v[2], v[3]);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
    if (s[b] != 0.f) atomicAdd(&colsum[c0 + b], s[b]);
}

// C[m][n] = sum_k fb[k][m] * fa[k][n], m over detector-B pixels, n over
// detector-A pixels; 128 x 128 tile per work-group, K tile 16, double-buffered
// LDS; thread (ty, tx) owns rows ty*4 + {0..3, 64..67} and columns
// tx*4 + {0..3, 64..67}.
__global__ __launch_bounds__(256) void k_sgemm_gamma(
    const float* __restrict__ fb, const float* __restrict__ fa, int64_t kpad, int64_t pb_pad,
    int64_t pa_pad, int64_t pa, int64_t pb, float nf, const float* __restrict__ sa,
    const float* __restrict__ sb, int layout, float* __restrict__ out) {
  __shared__ float sm[2][16][128];
  __shared__ float sn[2][16][128];
  const int t = threadIdx.x;
  const int ty = t >> 4, tx = t & 15;
  const int64_t tiles_m = pb_pad / 128;
  const int64_t tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int64_t m_base = tm * 128, n_base = tn * 128;

  // tile loader: 512 float4 per operand per K tile, two per thread
  const int l0 = t, l1 = t + 256;
  const int lr0 = l0 >> 5, lc0 = (l0 & 31) * 4;
  const int lr1 = l1 >> 5, lc1 = (l1 & 31) * 4;

  float acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0.f;

  const int64_t ktiles = kpad / 16;
  float4 rm0 = *reinterpret_cast<const float4*>(fb + int64_t(lr0) * pb_pad + m_base + lc0);
  float4 rm1 = *reinterpret_cast<const float4*>(fb + int64_t(lr1) * pb_pad + m_base + lc1);
  float4 rn0 = *reinterpret_cast<const float4*>(fa + int64_t(lr0) * pa_pad + n_base + lc0);
  float4 rn1 = *reinterpret_cast<const float4*>(fa + int64_t(lr1) * pa_pad + n_base + lc1);
  *reinterpret_cast<float4*>(&sm[0][lr0][lc0]) = rm0;
  *reinterpret_cast<float4*>(&sm[0][lr1][lc1]) = rm1;
  *reinterpret_cast<float4*>(&sn[0][lr0][lc0]) = rn0;
  *reinterpret_cast<float4*>(&sn[0][lr1][lc1]) = rn1;
  __syncthreads();

  for (int64_t kt = 0; kt < ktiles; ++kt) {
    const int cur = int(kt & 1);
    const bool more = kt + 1 < ktiles;
    if (more) {
      const int64_t k0 = (kt + 1) * 16;
      rm0 = *reinterpret_cast<const float4*>(fb + (k0 + lr0) * pb_pad + m_base + lc0);
      rm1 = *reinterpret_cast<const float4*>(fb + (k0 + lr1) * pb_pad + m_base + lc1);
      rn0 = *reinterpret_cast<const float4*>(fa + (k0 + lr0) * pa_pad + n_base + lc0);
      rn1 = *reinterpret_cast<const float4*>(fa + (k0 + lr1) * pa_pad + n_base + lc1);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float4 a0 = *reinterpret_cast<const float4*>(&sm[cur][k][ty * 4]);
      const float4 a1 = *reinterpret_cast<const float4*>(&sm[cur][k][64 + ty * 4]);
      const float4 b0 = *reinterpret_cast<const float4*>(&sn[cur][k][tx * 4]);
      const float4 b1 = *reinterpret_cast<const float4*>(&sn[cur][k][64 + tx * 4]);
      const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
      const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_fmaf(av[i], bv[j], acc[i][j]);
    }
    if (more) {
      const int nxt = cur ^ 1;
      *reinterpret_cast<float4*>(&sm[nxt][lr0][lc0]) = rm0;
      *reinterpret_cast<float4*>(&sm[nxt][lr1][lc1]) = rm1;
      *reinterpret_cast<float4*>(&sn[nxt][lr0][lc0]) = rn0;
      *reinterpret_cast<float4*>(&sn[nxt][lr1][lc1]) = rn1;
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t q = m_base + (i < 4 ? ty * 4 + i : 64 + ty * 4 + (i - 4));
    if (q >= pb) continue;
    const float mb = sb[q] / nf;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t p = n_base + (j < 4 ? tx * 4 + j : 64 + tx * 4 + (j - 4));
      if (p >= pa) continue;
      const float ma = sa[p] / nf;
      const float prod = ma * mb;
      const float mab = acc[i][j] / nf;
      const float gam = mab - prod;
      const int64_t idx = (layout == CPI_GAMMA_VIEW_MAJOR) ? q * pa + p : p * pb + q;
      out[idx] = gam;
    }
  }
}

}  // namespace

hipError_t unpack_f32(const uint8_t* frames, int fmt, int64_t n, int64_t npix, int64_t kpad,
                      int64_t cols_pad, float* out, float* colsum, hipStream_t s) {
  const int64_t gx = (cols_pad / 4 + 255) / 256;
  int64_t slices = (4096 + gx - 1) / gx;
  if (slices > kpad) slices = kpad;
  if (slices > 65535) slices = 65535;
  const int64_t fps = (kpad + slices - 1) / slices;
  slices = (kpad + fps - 1) / fps;
  hipLaunchKernelGGL(k_unpack_f32, dim3(unsigned(gx), unsigned(slices)), dim3(256), 0, s, frames,
                     fmt, n, npix, kpad, cols_pad, fps, out, colsum);
  return hipGetLastError();
}

hipError_t sgemm_gamma(const float* fb, const float* fa, int64_t kpad, int64_t pb_pad,
                       int64_t pa_pad, int64_t pa, int64_t pb, int64_t n, const float* sa,
                       const float* sb, int layout, float* out, hipStream_t s) {
  const int64_t nwg = (pb_pad / 128) * (pa_pad / 128);
  if (nwg <= 0 || nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sgemm_gamma, dim3(unsigned(nwg)), dim3(256), 0, s, fb, fa, kpad, pb_pad,
                     pa_pad, pa, pb, float(n), sa, sb, layout, out);
  return hipGetLastError();
}

}  // namespace cpi
