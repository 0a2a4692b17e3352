// Kernels of the learned denoiser: a convolutional encoder-decoder on BF16
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 sums), trained with Adam on
// FP32 master weights.
//
// Activations are NHWC bfloat16 tensors [B][H][W][C] (C innermost).  A
// convolution is an implicit GEMM: M = B*H*W output pixels, N = Cout output
// channels, K = KS*KS*Cin with k = tap*Cin + ci (tap = ky*KS + kx), zero
// padding of (KS-1)/2 pixels.  Weights are stored [Cout][Kpad] (K contiguous,
// zero-padded to a multiple of 32).  Every layer has Cin % 8 == 0 and
// Cout % 32 == 0 (narrower layers carry zero channels), so the 8 consecutive
// K values a lane feeds to one matrix-core op are 8 consecutive channels of
// one input pixel: one 16-byte load.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace cpi {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// Round to nearest even; NaN stays a (quiet) NaN.
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return uint16_t((u >> 16) | 0x40u);
  return uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// 2x2 max-pooling of 8 channels: elementwise maximum of the four 16-byte
// pieces at p, p + dx, p + dy, p + dy + dx, in that order (as k_maxpool)
__device__ __forceinline__ uint4 pool4(const uint16_t* p, int64_t dx, int64_t dy) {
  const uint4 v[4] = {*reinterpret_cast<const uint4*>(p), *reinterpret_cast<const uint4*>(p + dx),
                      *reinterpret_cast<const uint4*>(p + dy),
                      *reinterpret_cast<const uint4*>(p + dy + dx)};
  uint4 o;
  uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float m = bf2f(reinterpret_cast<const uint16_t*>(&v[0])[e]);
#pragma unroll
    for (int q = 1; q < 4; ++q) m = fmaxf(m, bf2f(reinterpret_cast<const uint16_t*>(&v[q])[e]));
    oh[e] = f2bf(m);
  }
  return o;
}

unsigned grid1(int64_t n, int threads = 256) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return unsigned(g);
}

// ---- convolution, forward and backward-data ---------------------------------
// A work-group of 4 waves covers 64*TM pixels x 16*TN output channels; wave w
// owns pixels [16*TM*w, 16*TM*(w+1)) of it and all 16*TN channels, as TM x TN
// tiles of 16 x 16.  Lane l holds pixel (or channel) l % 16 of a tile and K
// group l / 16 (8 consecutive K values: 8 channels of one input pixel at one
// tap).  The fragments of the next K step are loaded before the matrix-core
// ops of the current one.
template <int KS, int TM, int TN>
__global__ __launch_bounds__(256) void k_conv(NnConvArgs a) {
  constexpr int HALF = KS / 2;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t M = int64_t(a.B) * a.H * a.W;
  const int64_t m0 = int64_t(blockIdx.x) * (64 * TM) + wave * (16 * TM);
  const int n0 = blockIdx.y * (16 * TN);
  const int Cin = a.Cin;
  int py[TM], px[TM];
  const uint16_t* pbase[TM];
  bool pv[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int64_t m = m0 + 16 * i + r;
    pv[i] = m < M;
    const int64_t mm = pv[i] ? m : 0;
    px[i] = int(mm % a.W);
    py[i] = int((mm / a.W) % a.H);
    const int64_t b = mm / (int64_t(a.W) * a.H);
    pbase[i] = a.in + b * a.H * a.W * int64_t(Cin);
  }
  const uint16_t* wrow[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) wrow[j] = a.wk + int64_t(n0 + 16 * j + r) * a.Kpad + 8 * g;
  // this lane's K position (tap, ci) for k = kc + 8 g
  int tap = (8 * g) / Cin, ci = (8 * g) % Cin;

  uint4 a0[TM], b0[TN], a1[TM], b1[TN];
  auto load = [&](uint4 (&av)[TM], uint4 (&bv)[TN], int kc) {
    const int dy = tap / KS - HALF, dx = tap % KS - HALF;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int yy = py[i] + dy, xx = px[i] + dx;
      av[i] = make_uint4(0, 0, 0, 0);
      if (pv[i] && tap < KS * KS && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
        av[i] = *reinterpret_cast<const uint4*>(pbase[i] + (int64_t(yy) * a.W + xx) * Cin + ci);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) bv[j] = *reinterpret_cast<const uint4*>(wrow[j] + kc);
  };
  auto advance = [&]() {
    ci += 32;
    while (ci >= Cin) {
      ci -= Cin;
      ++tap;
    }
  };
  v4f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0, 0, 0, 0};
  auto mma = [&](const uint4 (&av)[TM], const uint4 (&bv)[TN]) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av[i]),
                                                            __builtin_bit_cast(v8bf, bv[j]),
                                                            acc[i][j], 0, 0, 0);
  };
  // two register stages: fragments of step kc + 32 load while step kc computes
  load(a0, b0, 0);
  for (int kc = 0; kc < a.Kpad; kc += 64) {
    const bool more1 = kc + 32 < a.Kpad;
    if (more1) {
      advance();
      load(a1, b1, kc + 32);
    }
    mma(a0, b0);
    if (!more1) break;
    if (kc + 64 < a.Kpad) {
      advance();
      load(a0, b0, kc + 64);
    }
    mma(a1, b1);
  }
  // element (pixel 4g + t, channel r) of each tile
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t m = m0 + 16 * i + 4 * g + t;
        const int n = n0 + 16 * j + r;
        if (m >= M) continue;
        float v = acc[i][j][t];
        if (a.bias) v += a.bias[n];
        if (a.relu && v < 0.0f) v = 0.0f;
        const int64_t o = m * a.Cout + n;
        if (a.mask && !(bf2f(a.mask[o]) > 0.0f)) v = 0.0f;
        if (a.out) a.out[o] = f2bf(v);
        if (a.out_f32) a.out_f32[o] = v;
      }
}

// ---- 3x3 convolution with LDS-staged tiles ------------------------------------
// For Cin % 32 == 0.  A work-group computes a block of TH = WM*TM output rows
// x 16 columns of one image and NT = WN*TN*16 output channels with 4 waves
// (WM x WN); wave (wm, wn) owns rows [wm*TM, (wm+1)*TM) (one 16-pixel
// fragment per row) and channels [wn*16*TN, (wn+1)*16*TN).  Per chunk of 32
// input channels the block's input pixels with their one-pixel halo
// ((TH + 2) x 18 pixels) are staged in LDS once; per phase of KY kernel rows
// (KY = 1 or 3) the weights of their taps for the NT channels are staged
// beside them, and those taps run from LDS.  Pixel and weight rows are padded
// to 40 elements (80 bytes) to spread LDS banks.
// MODE: 0 input and output as stored; 1 input read through the 2x2
// max-pool; 2 output split (dlow / dskip); 3 input concatenated (low).
template <int TM, int TN, int WM, int WN, int KY, int MODE>
__global__ __launch_bounds__(256) void k_conv3_lds(NnConvArgs a) {
  constexpr bool POOL = MODE == 1, SPLIT = MODE == 2, CAT = MODE == 3;
  constexpr int TH = WM * TM, TW = 16, NT = WN * TN * 16;
  constexpr int HW = TW + 2, HH = TH + 2;
  constexpr int PITCH = 40;  // elements per staged pixel / weight row
  static_assert(KY == 1 || KY == 3, "kernel rows per phase");
  __shared__ __attribute__((aligned(16))) uint16_t halo[HH * HW * PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t slab[3 * KY * NT * PITCH];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int wm = wave / WN, wn = wave % WN;
  const int cols = (a.W + TW - 1) / TW, rows = (a.H + TH - 1) / TH;
  int blk = blockIdx.x;
  const int bx = blk % cols;
  blk /= cols;
  const int by = blk % rows;
  const int b = blk / rows;
  const int x0 = bx * TW, y0 = by * TH;
  const int n0 = blockIdx.y * NT;
  const int Cin = a.Cin;
  // input channels [0, c_low) from the upsampled low-resolution tensor, the
  // rest from in (c_low = 0: all from in)
  const int Cs = Cin - a.c_low, Wl = a.W / 2;
  const uint16_t* img = a.in + int64_t(b) * a.H * a.W * Cs;
  const uint16_t* limg = a.low ? a.low + int64_t(b) * (a.H / 2) * Wl * a.c_low : nullptr;

  v4f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0, 0, 0, 0};

  // Phases p = (3 / KY) * chunk + kernel-row group.  The global loads of
  // phase p + 1 (the halo when a new chunk starts, and the weight slab) are
  // issued into registers before the matrix-core ops of phase p and written
  // to LDS after them.
  constexpr int PPC = 3 / KY;                          // phases per chunk
  constexpr int HQ = (HH * HW * 4 + 255) / 256;        // halo pieces per thread
  constexpr int SQ = (3 * KY * NT * 4 + 255) / 256;    // slab pieces per thread
  uint4 hreg[HQ], sreg[SQ];
  auto load_halo = [&](int c0) {
#pragma unroll
    for (int u = 0; u < HQ; ++u) {
      const int q = t + 256 * u;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (q < HH * HW * 4) {
        const int px = q >> 2, part = q & 3;
        const int hy = px / HW, hx = px % HW;
        const int yy = y0 + hy - 1, xx = x0 + hx - 1;
        if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) {
          if constexpr (POOL)
            v = pool4(a.in + ((int64_t(b) * 2 * a.H + 2 * yy) * 2 * a.W + 2 * xx) * Cin + c0 +
                          8 * part,
                      Cin, int64_t(2) * a.W * Cin);
          else
            v = (CAT && c0 < a.c_low)
                    ? *reinterpret_cast<const uint4*>(
                          limg + (int64_t(yy >> 1) * Wl + (xx >> 1)) * a.c_low + c0 + 8 * part)
                    : *reinterpret_cast<const uint4*>(img + (int64_t(yy) * a.W + xx) * Cs + c0 -
                                                      a.c_low + 8 * part);
        }
      }
      hreg[u] = v;
    }
  };
  auto store_halo = [&]() {
#pragma unroll
    for (int u = 0; u < HQ; ++u) {
      const int q = t + 256 * u;
      if (q < HH * HW * 4)
        *reinterpret_cast<uint4*>(&halo[(q >> 2) * PITCH + 8 * (q & 3)]) = hreg[u];
    }
  };
  auto load_slab = [&](int c0, int ky0) {
#pragma unroll
    for (int u = 0; u < SQ; ++u) {
      const int q = t + 256 * u;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (q < 3 * KY * NT * 4) {
        const int part = q & 3, row = q >> 2;  // row = (3 * kyi + kx) * NT + n
        const int tl = row / NT, n = row % NT;
        const int k = (ky0 * 3 + tl) * Cin + c0 + 8 * part;
        v = *reinterpret_cast<const uint4*>(a.wk + int64_t(n0 + n) * a.Kpad + k);
      }
      sreg[u] = v;
    }
  };
  auto store_slab = [&]() {
#pragma unroll
    for (int u = 0; u < SQ; ++u) {
      const int q = t + 256 * u;
      if (q < 3 * KY * NT * 4)
        *reinterpret_cast<uint4*>(&slab[(q >> 2) * PITCH + 8 * (q & 3)]) = sreg[u];
    }
  };

  const int phases = (Cin / 32) * PPC;
  load_halo(0);
  load_slab(0, 0);
  store_halo();
  store_slab();
  __syncthreads();
#pragma unroll 1
  for (int p = 0; p < phases; ++p) {
    const int ky0 = KY * (p % PPC);
    const bool next = p + 1 < phases;
    const int pn = p + 1, cn = 32 * (pn / PPC), kyn = KY * (pn % PPC);
    if (next) {
      if (kyn == 0) load_halo(cn);
      load_slab(cn, kyn);
    }
#pragma unroll
    for (int tl = 0; tl < 3 * KY; ++tl) {
      const int ky = ky0 + tl / 3, kx = tl % 3;
      uint4 av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        av[i] = *reinterpret_cast<const uint4*>(
            &halo[((wm * TM + i + ky) * HW + r + kx) * PITCH + 8 * g]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bv[j] = *reinterpret_cast<const uint4*>(
            &slab[(tl * NT + wn * 16 * TN + 16 * j + r) * PITCH + 8 * g]);
      // weights as the A operand (rows: channels), pixels as B (columns)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(v8bf, bv[j]), __builtin_bit_cast(v8bf, av[i]), acc[i][j], 0, 0,
              0);
    }
    if (next) {
      __syncthreads();  // every wave is done reading phase p's tiles
      if (kyn == 0) store_halo();
      store_slab();
      __syncthreads();
    }
  }
  // elements (column r of row wm*TM + i, channels 4g .. 4g + 3 of tile j):
  // four consecutive channels of one pixel per lane, stored together
  const int xx = x0 + r;
  if constexpr (SPLIT) {
    // split output: the 2x2 window of rows (i, i + 1) (TM even) and columns
    // (r, r ^ 1) (lanes r and r ^ 1)
    static_assert(TM % 2 == 0, "split output needs an even number of rows per wave");
    {
      const bool to_low = n0 < a.c1;  // the whole tile is on one side (c1 % NT == 0)
      const int C2 = a.Cout - a.c1;
#pragma unroll
      for (int i = 0; i < TM; i += 2) {
        const int yy = y0 + wm * TM + i;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int n = n0 + wn * 16 * TN + 16 * j + 4 * g;
          if (!to_low) {
#pragma unroll
            for (int di = 0; di < 2; ++di) {
              if (yy + di >= a.H || xx >= a.W) continue;
              uint2 ov;
              ov.x = uint32_t(f2bf(acc[i + di][j][0])) | (uint32_t(f2bf(acc[i + di][j][1])) << 16);
              ov.y = uint32_t(f2bf(acc[i + di][j][2])) | (uint32_t(f2bf(acc[i + di][j][3])) << 16);
              *reinterpret_cast<uint2*>(
                  a.dskip + ((int64_t(b) * a.H + yy + di) * a.W + xx) * C2 + (n - a.c1)) = ov;
            }
          } else {
            float sv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float v00 = bf2f(f2bf(acc[i][j][e])), v10 = bf2f(f2bf(acc[i + 1][j][e]));
              const float v01 = __shfl_xor(v00, 1), v11 = __shfl_xor(v10, 1);
              sv[e] = (v00 + v01) + (v10 + v11);
            }
            if ((r & 1) == 0 && yy < a.H && xx < a.W) {
              const int64_t lo =
                  ((int64_t(b) * (a.H / 2) + yy / 2) * (a.W / 2) + xx / 2) * a.c1 + n;
              uint2 mk = make_uint2(0x3F803F80u, 0x3F803F80u);  // 1.0 in every element
              if (a.low_mask) mk = *reinterpret_cast<const uint2*>(a.low_mask + lo);
              const uint16_t* mh = reinterpret_cast<const uint16_t*>(&mk);
              uint16_t o[4];
#pragma unroll
              for (int e = 0; e < 4; ++e) o[e] = bf2f(mh[e]) > 0.0f ? f2bf(sv[e]) : uint16_t(0);
              uint2 ov;
              ov.x = uint32_t(o[0]) | (uint32_t(o[1]) << 16);
              ov.y = uint32_t(o[2]) | (uint32_t(o[3]) << 16);
              *reinterpret_cast<uint2*>(a.dlow + lo) = ov;
            }
          }
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int yy = y0 + wm * TM + i;
    if (yy >= a.H || xx >= a.W) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wn * 16 * TN + 16 * j + 4 * g;
      const int64_t o = ((int64_t(b) * a.H + yy) * a.W + xx) * a.Cout + n;
      float v[4];
      uint2 mk = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
      if (a.mask) mk = *reinterpret_cast<const uint2*>(a.mask + o);
      const uint16_t* mh = reinterpret_cast<const uint16_t*>(&mk);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[e] = acc[i][j][e];
        if (a.bias) v[e] += a.bias[n + e];
        if (a.relu && v[e] < 0.0f) v[e] = 0.0f;
        if (a.mask && !(bf2f(mh[e]) > 0.0f)) v[e] = 0.0f;
      }
      if (a.out) {
        uint2 ov;
        ov.x = uint32_t(f2bf(v[0])) | (uint32_t(f2bf(v[1])) << 16);
        ov.y = uint32_t(f2bf(v[2])) | (uint32_t(f2bf(v[3])) << 16);
        *reinterpret_cast<uint2*>(a.out + o) = ov;
      }
      if (a.out_f32) *reinterpret_cast<float4*>(a.out_f32 + o) = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// ---- convolution, backward-weight -------------------------------------------
// dW[n][k] += sum over pixels m of dY[m][n] * X(m, k), X the implicit im2col of
// the input.  A work-group owns an NT x KT tile of dW (NT = 32 or 64 output
// channels, KT = 64 K values) and a range of pixels, taken 64 at a time: dY
// and X blocks are loaded with 16-byte loads and stored as they are in LDS
// ([pixel][channel]), and the matrix-core operands, whose K index is the
// pixel, are read with the transposing LDS loads of this part
// (ds_read_b64_tr_b16: within each 16 lanes, lane j receives element j % 4 of
// the 8-byte rows that lanes 4 k + j / 4 address, k = 0 .. 3; so when lane
// 4 k + q addresses pixel k, channels 4 q .. 4 q + 3, lane j gets channel j at
// four consecutive pixels).  NT = 64: wave w owns channels 32 (w & 1) +
// [0, 32) and K values (KT / 2) (w >> 1) + [0, KT / 2); NT = 32: all 32
// channels and K values (KT / 4) w + [0, KT / 4).  The work-group's tile goes
// to its pixel split's slot of the partial buffer (added to dW with FP32
// atomics when there is none).  Work-groups of the first K tile also sum
// their dY block over pixels into db (if given).
template <int KS, int NT, int KT>
__global__ __launch_bounds__(256) void k_conv_wgrad(NnWgradArgs a) {
  constexpr int HALF = KS / 2;
  constexpr int PB = 64;                 // pixels per block
  constexpr int KW = NT == 64 ? KT / 2 : KT / 4;  // K values per wave
  constexpr int NKB = KW / 16;                    // 16-wide K blocks per wave
  __shared__ __attribute__((aligned(16))) uint16_t ty[PB][NT + 8];
  __shared__ __attribute__((aligned(16))) uint16_t tx[PB][KT + 8];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int n0 = blockIdx.x * NT;
  const int kc = blockIdx.y * KT;
  const int64_t M = int64_t(a.B) * a.H * a.W;
  const int64_t per = ((M + gridDim.z - 1) / gridDim.z + PB - 1) / PB * PB;
  const int64_t mlo = int64_t(blockIdx.z) * per;
  const int64_t mhi = mlo + per < M ? mlo + per : M;
  const int Cin = a.Cin;
  const int K = KS * KS * Cin;
  const int nb0 = NT == 64 ? 32 * (wave & 1) : 0;
  const int kb0 = NT == 64 ? KW * (wave >> 1) : KW * wave;
  v4f acc[2][NKB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NKB; ++j) acc[i][j] = v4f{0, 0, 0, 0};
  const bool bias = a.db && blockIdx.y == 0;
  float bsum = 0.0f;
  // A block's loads all go out before any of its LDS writes, and the next
  // block's loads are issued before the current block's matrix-core ops.
  // Piece c covers pixel c % PB and channel group c / PB (16 bytes, stored
  // as loaded).
  constexpr int YQ = PB * (NT / 8) / 256;   // dY pieces per thread
  constexpr int XQ = PB * (KT / 8) / 256;   // X pieces per thread
  static_assert(YQ >= 1 && XQ >= 1, "tile too small for 256 threads");
  uint4 yv[YQ], xv[XQ];
  auto load = [&](int64_t mb) {
#pragma unroll
    for (int u = 0; u < YQ; ++u) {
      const int c = t + 256 * u;
      const int p = c % PB, q = c / PB;
      const int64_t m = mb + p;
      yv[u] = make_uint4(0, 0, 0, 0);
      if (m < mhi && n0 + 8 * q < a.Cout)
        yv[u] = *reinterpret_cast<const uint4*>(a.dy + m * a.Cout + n0 + 8 * q);
    }
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int c = t + 256 * u;
      const int p = c % PB, q = c / PB;
      const int64_t m = mb + p;
      const int k = kc + 8 * q;
      xv[u] = make_uint4(0, 0, 0, 0);
      if (m < mhi && k < K) {
        const int tap = k / Cin, ci = k - tap * Cin;
        const int x = int(m % a.W), y = int((m / a.W) % a.H);
        const int64_t b = m / (int64_t(a.W) * a.H);
        const int yy = y + tap / KS - HALF, xx = x + tap % KS - HALF;
        if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
          xv[u] = *reinterpret_cast<const uint4*>(a.in + ((b * a.H + yy) * a.W + xx) * Cin + ci);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < YQ; ++u) {
      const int c = t + 256 * u;
      *reinterpret_cast<uint4*>(&ty[c % PB][8 * (c / PB)]) = yv[u];
    }
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int c = t + 256 * u;
      *reinterpret_cast<uint4*>(&tx[c % PB][8 * (c / PB)]) = xv[u];
    }
  };
  typedef short v4s __attribute__((ext_vector_type(4)));
  typedef __attribute__((address_space(3))) v4s lds_v4s;
  // 8 K values (pixels 8 g .. 8 g + 7 of a 32-pixel step) of channel col0 +
  // r: two transposing reads, lane 4 k + q addressing pixel k (+ 4 in the
  // second), channels col0 + 4 q .. + 3
  auto frag = [&](const uint16_t* tile, int pitch, int p0, int col0) {
    const uint16_t* base = tile + (p0 + 8 * g + (r >> 2)) * pitch + col0 + 4 * (r & 3);
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(base));
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(base + 4 * pitch));
    typedef short v8s __attribute__((ext_vector_type(8)));
    const v8s v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(v8bf, v);
  };
  if (mlo < mhi) load(mlo);
  for (int64_t mb = mlo; mb < mhi; mb += PB) {
    store();
    __syncthreads();
    if (mb + PB < mhi) load(mb + PB);
    if (bias && t < NT)
      for (int p = 0; p < PB; ++p) bsum += bf2f(ty[p][t]);
#pragma unroll
    for (int s = 0; s < PB / 32; ++s) {
      v8bf av[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = frag(&ty[0][0], NT + 8, 32 * s, nb0 + 16 * i);
#pragma unroll
      for (int j = 0; j < NKB; ++j) {
        const v8bf bv = frag(&tx[0][0], KT + 8, 32 * s, kb0 + 16 * j);
#pragma unroll
        for (int i = 0; i < 2; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv, acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // element (n = nb0 + 16 i + 4g + e, k = kb0 + 16 j + r)
  float* pz = a.part ? a.part + int64_t(blockIdx.z) * (int64_t(a.Cout) * K + a.Cout) : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NKB; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + nb0 + 16 * i + 4 * g + e;
        const int k = kc + kb0 + 16 * j + r;
        if (n < a.Cout && k < K) {
          if (pz)
            __builtin_nontemporal_store(acc[i][j][e], &pz[int64_t(n) * K + k]);
          else
            atomicAdd(&a.dw[int64_t(n) * K + k], acc[i][j][e]);
        }
      }
  if (bias && t < NT && n0 + t < a.Cout) {
    if (pz)
      __builtin_nontemporal_store(bsum, &pz[int64_t(a.Cout) * K + n0 + t]);
    else
      atomicAdd(&a.db[n0 + t], bsum);
  }
}

// ---- 3x3 convolution, backward-weight, all taps per work-group --------------
// dW[n][tap * Cin + ci] = sum over pixels (y, x) of dY[y][x][n] *
// X[y + ky - 1][x + kx - 1][ci], tap = 3 ky + kx.  A work-group owns NT
// output channels x one slice of 32 input channels x all nine taps, and walks
// a range of pixel blocks of R rows x TW columns.  Per block, the dY block
// ([pixel][channel]) and its input halo ((R + 2) x (TW + 2) pixels of the 32
// channels, zero outside the image) are staged in LDS once, and all nine taps
// read the one halo at shifted offsets, so each input pixel is fetched about
// once per slice instead of once per tap.  The matrix-core K index is the
// pixel: both operands come from the transposing LDS reads
// (ds_read_b64_tr_b16; lane 4 k + q addresses pixel p + k, channels
// c + 4 q .. + 3, and lane j receives channel c + j at pixels p .. p + 3).
// K slots 8 g .. 8 g + 7 of a 32-pixel step hold pixels 4 g .. 4 g + 3 and
// 16 + 4 g .. + 3, so the eight pixels that half a wave reads in one go are
// consecutive; with row pitches of an odd multiple of 32 bytes they cover all
// 64 LDS banks once.  Wave w takes input channels 16 (w & 1) + [0, 16); for
// NT = 64 it takes output channels 32 (w >> 1) + [0, 32) and every step, for
// NT = 32 all 32 channels and the steps of parity w >> 1.  A wave's 18 tiles
// (2 channel tiles x 9 taps) go to the pixel split's slot of the partial
// buffer (added to dW with FP32 atomics when there is none); the bias
// gradient is summed from the dY operands of the waves on input channels
// 0 .. 15 of the first slice.
template <int NT, int TW, int R>
__global__ __launch_bounds__(256) void k_conv3_wgrad(NnWgradArgs a) {
  constexpr int PXB = TW * R;             // pixels per block
  constexpr int STEPS = PXB / 32;         // 32-pixel matrix-core steps per block
  constexpr int PY = NT + 16;             // dY row pitch (elements): 96 or 160 bytes
  constexpr int PX = 48;                  // halo row pitch (elements): 96 bytes
  constexpr int HW = TW + 2, HP = (R + 2) * HW;
  static_assert(PXB % 64 == 0 && TW % 16 == 0, "block shape");
  static_assert(NT == 32 || NT == 64, "channel tile");
  // the dY block, then the halo; reused at the end (NT = 32) to combine the
  // two step parities: [9][32][RP] floats of dW, then 32 floats of db
  constexpr int TY = PXB * PY, TX = HP * PX, RP = 36;
  static_assert(NT == 64 || (9 * 32 * RP + 32) * 4 <= (TY + TX) * 2, "reduction space");
  __shared__ __attribute__((aligned(16))) uint16_t lds[TY + TX];
  uint16_t* const ty = lds;
  uint16_t* const tx = lds + TY;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int ct = wave & 1;
  const int nt0 = NT == 64 ? 2 * (wave >> 1) : 0;
  const int par = NT == 64 ? 0 : wave >> 1;
  const int n0 = blockIdx.x * NT, c0 = blockIdx.y * 32;
  const int Cin = a.Cin, K = 9 * Cin;
  const int bx = (a.W + TW - 1) / TW, by = (a.H + R - 1) / R;
  const int64_t nb = int64_t(a.B) * bx * by;
  const int64_t per = (nb + gridDim.z - 1) / gridDim.z;
  const int64_t blo = int64_t(blockIdx.z) * per;
  const int64_t bhi = blo + per < nb ? blo + per : nb;
  const bool bias = a.db && blockIdx.y == 0 && ct == 0;

  v4f acc[9][2];
#pragma unroll
  for (int u = 0; u < 9; ++u) acc[u][0] = acc[u][1] = v4f{0, 0, 0, 0};
  float bsum[2] = {0.0f, 0.0f};

  // staging: dY piece c = (pixel c / (NT / 8), channels 8 (c % (NT / 8)));
  // halo piece c = (halo pixel c / 4, channels 8 (c % 4))
  constexpr int YQ = PXB * NT / 8 / 256;
  constexpr int XQ = (HP * 4 + 255) / 256;
  static_assert(YQ * 256 == PXB * NT / 8, "dY pieces");
  uint4 yv[YQ], xv[XQ];
  auto load = [&](int64_t blk) {
    const int ix = int(blk % bx);
    const int64_t rest = blk / bx;
    const int iy = int(rest % by);
    const int64_t b = rest / by;
    const int x0 = ix * TW, y0 = iy * R;
#pragma unroll
    for (int u = 0; u < YQ; ++u) {
      const int c = t + 256 * u;
      const int px = c / (NT / 8), part = c % (NT / 8);
      const int y = y0 + px / TW, x = x0 + px % TW;
      yv[u] = make_uint4(0, 0, 0, 0);
      if (y < a.H && x < a.W)
        yv[u] = *reinterpret_cast<const uint4*>(a.dy + ((b * a.H + y) * a.W + x) * a.Cout + n0 +
                                                8 * part);
    }
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int c = t + 256 * u;
      const int hp = c >> 2, part = c & 3;
      const int y = y0 + hp / HW - 1, x = x0 + hp % HW - 1;
      xv[u] = make_uint4(0, 0, 0, 0);
      if (c < HP * 4 && y >= 0 && y < a.H && x >= 0 && x < a.W && a.pool_in)
        xv[u] = pool4(a.in + ((b * 2 * a.H + 2 * y) * 2 * a.W + 2 * x) * Cin + c0 + 8 * part, Cin,
                      int64_t(2) * a.W * Cin);
      else if (c < HP * 4 && y >= 0 && y < a.H && x >= 0 && x < a.W)
        xv[u] = c0 < a.c_low
                    ? *reinterpret_cast<const uint4*>(
                          a.low + ((b * (a.H / 2) + (y >> 1)) * (a.W / 2) + (x >> 1)) * a.c_low +
                          c0 + 8 * part)
                    : *reinterpret_cast<const uint4*>(
                          a.in + ((b * a.H + y) * a.W + x) * (Cin - a.c_low) + c0 - a.c_low +
                          8 * part);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < YQ; ++u) {
      const int c = t + 256 * u;
      *reinterpret_cast<uint4*>(&ty[(c / (NT / 8)) * PY + 8 * (c % (NT / 8))]) = yv[u];
    }
#pragma unroll
    for (int u = 0; u < XQ; ++u) {
      const int c = t + 256 * u;
      if (c < HP * 4) *reinterpret_cast<uint4*>(&tx[(c >> 2) * PX + 8 * (c & 3)]) = xv[u];
    }
  };
  typedef short v4s __attribute__((ext_vector_type(4)));
  typedef short v8s __attribute__((ext_vector_type(8)));
  typedef __attribute__((address_space(3))) v4s lds_v4s;
  // lane parts of the addresses: pixel 4 g + (r >> 2), channels 4 (r & 3)
  const uint16_t* ybase = ty + (4 * g + (r >> 2)) * PY + 16 * nt0 + 4 * (r & 3);
  const uint16_t* xbase = tx + (4 * g + (r >> 2)) * PX + 16 * ct + 4 * (r & 3);
  auto pair = [](const uint16_t* lo, const uint16_t* hi) {
    const v4s u = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)lo);
    const v4s v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)hi);
    const v8s w = {u[0], u[1], u[2], u[3], v[0], v[1], v[2], v[3]};
    return __builtin_bit_cast(v8bf, w);
  };

  if (blo < bhi) load(blo);
#pragma unroll 1
  for (int64_t blk = blo; blk < bhi; ++blk) {
    store();
    __syncthreads();
    if (blk + 1 < bhi) load(blk + 1);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      if (NT == 32 && (s & 1) != par) continue;
      // block pixel 32 s + 16 h + lane part: row (32 s + 16 h) / TW, column
      // (32 s + 16 h) % TW + lane part (a 16-pixel run never crosses a row)
      const int p0 = 32 * s, p1 = 32 * s + 16;
      v8bf av[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        av[i] = pair(ybase + p0 * PY + 16 * i, ybase + p1 * PY + 16 * i);
        if (bias) {
          const v8s e = __builtin_bit_cast(v8s, av[i]);
#pragma unroll
          for (int j = 0; j < 8; ++j) bsum[i] += bf2f(uint16_t(e[j]));
        }
      }
      const int h0 = (p0 / TW) * HW + p0 % TW, h1 = (p1 / TW) * HW + p1 % TW;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int o = ky * HW + kx;
          const v8bf bv = pair(xbase + (h0 + o) * PX, xbase + (h1 + o) * PX);
#pragma unroll
          for (int i = 0; i < 2; ++i)
            acc[3 * ky + kx][i] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv, acc[3 * ky + kx][i], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  // element (n = n0 + 16 (nt0 + i) + 4 g + e, ci = c0 + 16 ct + r) of tap u
  float* pz = a.part ? a.part + int64_t(blockIdx.z) * (int64_t(a.Cout) * K + a.Cout) : nullptr;
  float bv[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    bv[i] = bsum[i];
    bv[i] += __shfl_xor(bv[i], 16);
    bv[i] += __shfl_xor(bv[i], 32);
  }
  if (NT == 64) {
#pragma unroll
    for (int u = 0; u < 9; ++u)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int n = n0 + 16 * (nt0 + i) + 4 * g + e;
          const int64_t o = int64_t(n) * K + u * Cin + c0 + 16 * ct + r;
          if (pz)
            __builtin_nontemporal_store(acc[u][i][e], &pz[o]);
          else
            atomicAdd(&a.dw[o], acc[u][i][e]);
        }
  } else {
    // the waves of parity 1 add their tiles to those of parity 0 in LDS (the
    // loop's last barrier has freed it), then the work-group stores the
    // 32 x 9 x 32 tile with coalesced writes
    float* red = reinterpret_cast<float*>(lds);
    float* rb = red + 9 * 32 * RP;
    if (par == 0) {
#pragma unroll
      for (int u = 0; u < 9; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            red[(u * 32 + 16 * i + 4 * g + e) * RP + 16 * ct + r] = acc[u][i][e];
      if (bias && g == 0) rb[r] = bv[0], rb[16 + r] = bv[1];
    }
    __syncthreads();
    if (par == 1) {
#pragma unroll
      for (int u = 0; u < 9; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            red[(u * 32 + 16 * i + 4 * g + e) * RP + 16 * ct + r] += acc[u][i][e];
      if (bias && g == 0) rb[r] += bv[0], rb[16 + r] += bv[1];
    }
    __syncthreads();
    for (int q = t; q < 9 * 32 * 32; q += 256) {
      const int u = q >> 10, n = (q >> 5) & 31, ci = q & 31;
      const float v = red[(u * 32 + n) * RP + ci];
      const int64_t o = int64_t(n0 + n) * K + u * Cin + c0 + ci;
      if (pz)
        __builtin_nontemporal_store(v, &pz[o]);
      else
        atomicAdd(&a.dw[o], v);
    }
    if (bias && par == 0 && g == 0) bv[0] = rb[r], bv[1] = rb[16 + r];
  }
  if (bias && par == 0 && g == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int n = n0 + 16 * (nt0 + i) + r;
      if (pz)
        __builtin_nontemporal_store(bv[i], &pz[int64_t(a.Cout) * K + n]);
      else
        atomicAdd(&a.db[n], bv[i]);
    }
  }
}

// dw[i] += sum over splits z of part[z][i] (i < nw), db[i - nw] += the same
// for the bias slots (db non-null).  Rows are nw + cout floats, a multiple
// of 4, and part is 16-byte aligned.  A work-group takes 64 consecutive
// elements as 16 float4 columns; thread (slot, l) sums splits slot,
// slot + 16, ... of column l in that order, and thread e < 64 then adds the
// 16 slot sums of element e in slot order: a fixed order, whatever the
// scheduling.
// scx > 0: the nw weight slots are dense (n, tap) pairs of a 3x3 layer with
// one input channel used of scx, added to dw[n][tap * scx].
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int splits,
                                                      int64_t nw, int cout,
                                                      float* __restrict__ dw,
                                                      float* __restrict__ db, int scx = 0) {
  __shared__ v4f red[256];
  const int t = threadIdx.x, l = t & 15, slot = t >> 4;
  const int64_t stride = nw + cout, n = db ? stride : nw, st4 = stride / 4;
  for (int64_t i0 = int64_t(blockIdx.x) * 64; i0 < n; i0 += int64_t(gridDim.x) * 64) {
    const int64_t i = i0 + 4 * l;
    v4f s = {0.0f, 0.0f, 0.0f, 0.0f};
    if (i < n) {
      const v4f* q = reinterpret_cast<const v4f*>(part + i);
      int z = slot;
      for (; z + 48 < splits; z += 64) {
        const v4f v0 = __builtin_nontemporal_load(q + z * st4);
        const v4f v1 = __builtin_nontemporal_load(q + (z + 16) * st4);
        const v4f v2 = __builtin_nontemporal_load(q + (z + 32) * st4);
        const v4f v3 = __builtin_nontemporal_load(q + (z + 48) * st4);
        s += v0;
        s += v1;
        s += v2;
        s += v3;
      }
      for (; z < splits; z += 16) s += __builtin_nontemporal_load(q + z * st4);
    }
    red[t] = s;
    __syncthreads();
    if (t < 64 && i0 + t < n) {
      const float* rf = reinterpret_cast<const float*>(red);
      float tot = 0.0f;
      for (int k = 0; k < 16; ++k) tot += rf[4 * (16 * k + (t >> 2)) + (t & 3)];
      const int64_t i = i0 + t;
      if (i >= nw)
        db[i - nw] += tot;
      else if (scx > 0)
        dw[(i / 9) * 9 * scx + (i % 9) * scx] += tot;
      else
        dw[i] += tot;
    }
    __syncthreads();
  }
}

// db[n] += sum over pixels of dY[m][n]
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t* __restrict__ dy, int64_t M,
                                                   int C, float* __restrict__ db) {
  const int n = blockIdx.y * 64 + (threadIdx.x & 63);
  const int row = threadIdx.x >> 6;
  float s = 0.0f;
  if (n < C)
    for (int64_t m = int64_t(blockIdx.x) * 4 + row; m < M; m += int64_t(gridDim.x) * 4)
      s += bf2f(dy[m * C + n]);
  __shared__ float red[4][64];
  red[row][threadIdx.x & 63] = s;
  __syncthreads();
  if (row == 0 && n < C) atomicAdd(&db[n], red[0][threadIdx.x] + red[1][threadIdx.x] +
                                               red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// FP32 master weights [Cout][ks*ks][Cin] -> BF16 [Cout][kpad] (forward) and
// the flipped, transposed [Cin][kpad_t] with K' = tap'*Cout + co, tap' =
// ks*ks-1-tap (backward-data).
__global__ __launch_bounds__(256) void k_pack_weights(const float* __restrict__ w, int Cout,
                                                      int Cin, int ks, uint16_t* __restrict__ wf,
                                                      int kpad, uint16_t* __restrict__ wt,
                                                      int kpad_t) {
  const int taps = ks * ks;
  const int64_t nf = int64_t(Cout) * kpad, nt = wt ? int64_t(Cin) * kpad_t : 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nf + nt;
       i += int64_t(gridDim.x) * 256) {
    if (i < nf) {
      const int co = int(i / kpad), k = int(i % kpad);
      wf[i] = k < taps * Cin ? f2bf(w[int64_t(co) * taps * Cin + k]) : uint16_t(0);
    } else {
      const int64_t j = i - nf;
      const int ci = int(j / kpad_t), k = int(j % kpad_t);
      uint16_t v = 0;
      if (k < taps * Cout) {
        const int tp = k / Cout, co = k % Cout;
        v = f2bf(w[(int64_t(co) * taps + (taps - 1 - tp)) * Cin + ci]);
      }
      wt[j] = v;
    }
  }
}

// The same packing for every layer of a network in one launch; element i of
// the concatenated packed arrays belongs to the last layer whose begin <= i.
__global__ __launch_bounds__(256) void k_pack_all(const float* __restrict__ params,
                                                  uint16_t* __restrict__ packed, NnPackTable tab) {
  // one grid row per layer; every per-layer index fits 32 bits
  const NnPackLayer& L = tab.layer[blockIdx.y];
  const int taps = L.ks * L.ks;
  const float* w = params + L.w_off;
  const int nf = L.cout * L.kpad;
  const int n = nf + (L.transposed ? L.cin * L.kpad_t : 0);
  for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
    if (j < nf) {
      const int co = j / L.kpad, k = j - co * L.kpad;
      packed[L.wf_off + j] = k < taps * L.cin ? f2bf(w[co * taps * L.cin + k]) : uint16_t(0);
    } else {
      const int jt = j - nf;
      const int ci = jt / L.kpad_t, k = jt - ci * L.kpad_t;
      uint16_t v = 0;
      if (k < taps * L.cout) {
        const int tp = k / L.cout, co = k - tp * L.cout;
        v = f2bf(w[(co * taps + (taps - 1 - tp)) * L.cin + ci]);
      }
      packed[L.wt_off + jt] = v;
    }
  }
}

// ---- pooling, upsampling, concatenation, masks ------------------------------
__global__ __launch_bounds__(256) void k_maxpool(const uint16_t* __restrict__ in, int B, int H,
                                                 int W, int C, uint16_t* __restrict__ out) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t n = int64_t(B) * Ho * Wo * C;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int c = int(i % C);
    const int64_t p = i / C;
    const int x = int(p % Wo), y = int((p / Wo) % Ho), b = int(p / (int64_t(Wo) * Ho));
    const uint16_t* s = in + ((int64_t(b) * H + 2 * y) * W + 2 * x) * C + c;
    float m = bf2f(s[0]);
    m = fmaxf(m, bf2f(s[C]));
    m = fmaxf(m, bf2f(s[int64_t(W) * C]));
    m = fmaxf(m, bf2f(s[int64_t(W) * C + C]));
    out[i] = f2bf(m);
  }
}

// Gradient of the 2 x 2 maximum: to the first position (in window order)
// holding the maximum.
__global__ __launch_bounds__(256) void k_maxpool_bwd(const uint16_t* __restrict__ in, int B,
                                                     int H, int W, int C,
                                                     const uint16_t* __restrict__ dout,
                                                     uint16_t* __restrict__ din) {
  const int Ho = H / 2, Wo = W / 2;
  const int64_t n = int64_t(B) * Ho * Wo * C;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int c = int(i % C);
    const int64_t p = i / C;
    const int x = int(p % Wo), y = int((p / Wo) % Ho), b = int(p / (int64_t(Wo) * Ho));
    const int64_t base = ((int64_t(b) * H + 2 * y) * W + 2 * x) * C + c;
    const int64_t off[4] = {0, C, int64_t(W) * C, int64_t(W) * C + C};
    int best = 0;
    float m = bf2f(in[base]);
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      const float v = bf2f(in[base + off[q]]);
      if (v > m) {
        m = v;
        best = q;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) din[base + off[q]] = q == best ? dout[i] : uint16_t(0);
  }
}

// nearest 2x upsampling and its gradient (sum of the 4 copies, zeroed where
// mask <= 0 if a mask is given)
__global__ __launch_bounds__(256) void k_upsample(const uint16_t* __restrict__ in, int B, int H,
                                                  int W, int C, uint16_t* __restrict__ out) {
  const int64_t n = int64_t(B) * 4 * H * W * C;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int c = int(i % C);
    const int64_t p = i / C;
    const int x = int(p % (2 * W)), y = int((p / (2 * W)) % (2 * H)), b = int(p / (4 * int64_t(W) * H));
    out[i] = in[((int64_t(b) * H + y / 2) * W + x / 2) * C + c];
  }
}

__global__ __launch_bounds__(256) void k_upsample_bwd(const uint16_t* __restrict__ dout, int B,
                                                      int H, int W, int C,
                                                      const uint16_t* __restrict__ mask,
                                                      uint16_t* __restrict__ din) {
  const int64_t n = int64_t(B) * H * W * C;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int c = int(i % C);
    const int64_t p = i / C;
    const int x = int(p % W), y = int((p / W) % H), b = int(p / (int64_t(W) * H));
    const int64_t base = ((int64_t(b) * 2 * H + 2 * y) * 2 * W + 2 * x) * C + c;
    const float s = (bf2f(dout[base]) + bf2f(dout[base + C])) +
                    (bf2f(dout[base + int64_t(2 * W) * C]) + bf2f(dout[base + int64_t(2 * W) * C + C]));
    din[i] = (mask && !(bf2f(mask[i]) > 0.0f)) ? uint16_t(0) : f2bf(s);
  }
}

// out[p] = [a[p] (C1 channels), b[p] (C2 channels)]; split is the inverse.
__global__ __launch_bounds__(256) void k_concat(const uint16_t* __restrict__ a,
                                                const uint16_t* __restrict__ b, int64_t P, int C1,
                                                int C2, uint16_t* __restrict__ out, int split) {
  const int C = C1 + C2;
  const int64_t n = P * C;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int64_t p = i / C;
    const int c = int(i % C);
    if (!split) {
      out[i] = c < C1 ? a[p * C1 + c] : b[p * C2 + (c - C1)];
    } else {
      // here `out` is the concatenated gradient and a, b receive its parts
      uint16_t* da = const_cast<uint16_t*>(a);
      uint16_t* db = const_cast<uint16_t*>(b);
      if (c < C1)
        da[p * C1 + c] = out[i];
      else
        db[p * C2 + (c - C1)] = out[i];
    }
  }
}

// out[b][y][x] = [up[b][y/2][x/2] (C1 channels), skip[b][y][x] (C2 channels)]
// for the 2H x 2W output (nearest 2x upsampling of the H x W input, then
// concatenation); 8 channels (16 bytes) per thread.  C1 % 8 == C2 % 8 == 0.
__global__ __launch_bounds__(256) void k_upcat(const uint16_t* __restrict__ low,
                                               const uint16_t* __restrict__ skip, int B, int H,
                                               int W, int C1, int C2,
                                               uint16_t* __restrict__ out) {
  const int q1 = C1 / 8, qt = (C1 + C2) / 8;
  const int64_t n = int64_t(B) * 4 * H * W * qt;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const int q = int(i % qt);
    const int64_t p = i / qt;  // output pixel
    uint4 v;
    if (q < q1) {
      const int x = int(p % (2 * W)), y = int((p / (2 * W)) % (2 * H));
      const int64_t b = p / (4 * int64_t(W) * H);
      v = *reinterpret_cast<const uint4*>(low + ((b * H + y / 2) * W + x / 2) * C1 + 8 * q);
    } else {
      v = *reinterpret_cast<const uint4*>(skip + p * C2 + 8 * (q - q1));
    }
    *reinterpret_cast<uint4*>(out + i * 8) = v;
  }
}

// Gradient of k_upcat: dskip = the last C2 channels of d; dlow[b][y][x][c] =
// sum of d over the 4 output pixels of (y, x) in channel c < C1 (FP32, then
// bfloat16), zeroed where mask <= 0 (nullable).  One thread per 8 channels of
// one output pixel of either part.
__global__ __launch_bounds__(256) void k_upcat_grad(const uint16_t* __restrict__ d, int B, int H,
                                                    int W, int C1, int C2,
                                                    const uint16_t* __restrict__ mask,
                                                    uint16_t* __restrict__ dlow,
                                                    uint16_t* __restrict__ dskip) {
  const int q1 = C1 / 8, q2 = C2 / 8, qt = q1 + q2;
  const int64_t nlow = int64_t(B) * H * W * q1;
  const int64_t nskip = int64_t(B) * 4 * H * W * q2;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nlow + nskip;
       i += int64_t(gridDim.x) * 256) {
    if (i < nlow) {
      const int q = int(i % q1);
      const int64_t p = i / q1;  // low-resolution pixel
      const int x = int(p % W), y = int((p / W) % H);
      const int64_t b = p / (int64_t(W) * H);
      const int64_t o00 = ((b * 2 * H + 2 * y) * 2 * W + 2 * x) * (C1 + C2) + 8 * q;
      const int64_t row = int64_t(2 * W) * (C1 + C2);
      const uint4 v0 = *reinterpret_cast<const uint4*>(d + o00);
      const uint4 v1 = *reinterpret_cast<const uint4*>(d + o00 + (C1 + C2));
      const uint4 v2 = *reinterpret_cast<const uint4*>(d + o00 + row);
      const uint4 v3 = *reinterpret_cast<const uint4*>(d + o00 + row + (C1 + C2));
      const uint16_t* h0 = reinterpret_cast<const uint16_t*>(&v0);
      const uint16_t* h1 = reinterpret_cast<const uint16_t*>(&v1);
      const uint16_t* h2 = reinterpret_cast<const uint16_t*>(&v2);
      const uint16_t* h3 = reinterpret_cast<const uint16_t*>(&v3);
      uint4 mv = make_uint4(0x3F80u * 0x10001u, 0x3F80u * 0x10001u, 0x3F80u * 0x10001u,
                            0x3F80u * 0x10001u);  // 1.0 in every lane of the mask
      if (mask) mv = *reinterpret_cast<const uint4*>(mask + p * C1 + 8 * q);
      const uint16_t* hm = reinterpret_cast<const uint16_t*>(&mv);
      uint4 r;
      uint16_t* hr = reinterpret_cast<uint16_t*>(&r);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float s = (bf2f(h0[e]) + bf2f(h1[e])) + (bf2f(h2[e]) + bf2f(h3[e]));
        hr[e] = bf2f(hm[e]) > 0.0f ? f2bf(s) : uint16_t(0);
      }
      *reinterpret_cast<uint4*>(dlow + p * C1 + 8 * q) = r;
    } else {
      const int64_t j = i - nlow;
      const int q = int(j % q2);
      const int64_t p = j / q2;  // output pixel
      *reinterpret_cast<uint4*>(dskip + p * C2 + 8 * q) =
          *reinterpret_cast<const uint4*>(d + p * (C1 + C2) + 8 * (q1 + q));
    }
  }
}

// x = (x + add) where mask > 0, 0 elsewhere (add and mask nullable)
__global__ __launch_bounds__(256) void k_add_mask(uint16_t* __restrict__ x,
                                                  const uint16_t* __restrict__ add,
                                                  const uint16_t* __restrict__ mask, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    float v = bf2f(x[i]);
    if (add) v += bf2f(add[i]);
    if (mask && !(bf2f(mask[i]) > 0.0f)) v = 0.0f;
    x[i] = f2bf(v);
  }
}

// ---- loss and optimiser ------------------------------------------------------
// Mean squared error of the prediction z = y[p][0] + res[p] (y with C
// channels per pixel, res nullable) against t over P pixels:
// loss += sum (z - t)^2 / P; dy = 2 (z - t) / P in channel 0, 0 elsewhere.
// The first 3x3 layer, whose input has one channel used of cx stored (the
// others zero): out[p][n] = relu(b[n] + sum over taps of w[n][tap] x[p + tap]
// (channel 0, zero padding)) for 32 output channels, w the packed weights
// (w[n][tap] at wk[n * kpad + tap * cx]); products of bfloat16 values summed
// in FP32 in tap order.
__global__ __launch_bounds__(256) void k_in1_fwd(const uint16_t* __restrict__ x, int B, int H,
                                                 int W, int cx, const uint16_t* __restrict__ wk,
                                                 int kpad, const float* __restrict__ bias,
                                                 uint16_t* __restrict__ out) {
  // weights as [tap][channel] (four channels per 16-byte read), bias after
  __shared__ __attribute__((aligned(16))) float ws[10 * 32];
  const int t = threadIdx.x;
  for (int q = t; q < 32 * 9; q += 256) ws[(q % 9) * 32 + q / 9] = bf2f(wk[(q / 9) * kpad + (q % 9) * cx]);
  if (t < 32) ws[9 * 32 + t] = bias ? bias[t] : 0.0f;
  __syncthreads();
  const v4f* w4 = reinterpret_cast<const v4f*>(ws);
  const int P = B * H * W;  // < 2^26 (the network's shape check)
  // two pixels per thread: p and p + half of the grid's stride
  const int stride = gridDim.x * 512;
  for (int p0 = blockIdx.x * 512 + t; p0 < P; p0 += stride) {
    int pp[2] = {p0, p0 + 256};
    float v[2][9];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int p = pp[u] < P ? pp[u] : p0;
      const int row = p / W, xx = p - row * W, yy = row % H;
      const int img = p - (yy * W + xx);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int y = yy + tap / 3 - 1, xc = xx + tap % 3 - 1;
        v[u][tap] = (y >= 0 && y < H && xc >= 0 && xc < W)
                        ? bf2f(x[int64_t(img + y * W + xc) * cx])
                        : 0.0f;
      }
    }
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      v4f acc[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) acc[u][0] = acc[u][1] = v4f{0, 0, 0, 0};
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const v4f wa = w4[tap * 8 + 2 * q], wb = w4[tap * 8 + 2 * q + 1];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            acc[u][0][e] = __builtin_fmaf(wa[e], v[u][tap], acc[u][0][e]);
            acc[u][1][e] = __builtin_fmaf(wb[e], v[u][tap], acc[u][1][e]);
          }
      }
      const v4f ba = w4[72 + 2 * q], bb = w4[72 + 2 * q + 1];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (pp[u] >= P) continue;
        uint4 o;
        uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float ra = acc[u][0][e] + ba[e], rb = acc[u][1][e] + bb[e];
          oh[e] = f2bf(ra < 0.0f ? 0.0f : ra);
          oh[4 + e] = f2bf(rb < 0.0f ? 0.0f : rb);
        }
        *reinterpret_cast<uint4*>(out + int64_t(pp[u]) * 32 + 8 * q) = o;
      }
    }
  }
}

// Weight and bias gradients of that layer: dW[n][tap * cx] = sum over pixels
// of dy[p][n] x[p + tap] (channel 0) and db[n] = sum of dy[p][n], as one row
// of 320 partial sums per work-group (n * 9 + tap, then the 32 bias slots).
// Thread t takes channels 8 (t & 3) .. + 7 of every 64th pixel of the
// work-group's range; the 64 threads of one channel group are then summed
// through LDS in thread order (two rounds of 40 of the 80 sums).
__global__ __launch_bounds__(256) void k_in1_wgrad(const uint16_t* __restrict__ x, int B, int H,
                                                   int W, int cx, const uint16_t* __restrict__ dy,
                                                   float* __restrict__ part) {
  __shared__ float red[40][257];
  __shared__ float fin[4 * 80];
  const int t = threadIdx.x;
  const int q = t & 3;
  const int P = B * H * W;  // < 2^26 (the network's shape check)
  const int per = (P + gridDim.x - 1) / gridDim.x;
  const int plo = blockIdx.x * per;
  const int phi = plo + per < P ? plo + per : P;
  float acc[80];
#pragma unroll
  for (int k = 0; k < 80; ++k) acc[k] = 0.0f;
#pragma unroll 4
  for (int p = plo + (t >> 2); p < phi; p += 64) {
    const int row = p / W, xx = p - row * W, yy = row % H;
    const int img = p - (yy * W + xx);
    float v[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int y = yy + tap / 3 - 1, xc = xx + tap % 3 - 1;
      v[tap] = (y >= 0 && y < H && xc >= 0 && xc < W) ? bf2f(x[int64_t(img + y * W + xc) * cx])
                                                      : 0.0f;
    }
    const uint4 d4 = *reinterpret_cast<const uint4*>(dy + int64_t(p) * 32 + 8 * q);
    const uint16_t* dh = reinterpret_cast<const uint16_t*>(&d4);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float d = bf2f(dh[e]);
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) acc[e * 9 + tap] = __builtin_fmaf(d, v[tap], acc[e * 9 + tap]);
      acc[72 + e] += d;
    }
  }
  // threads t = 4 m + q (m = 0 .. 63) share channel group q: sum 40 of the
  // 80 accumulators per round, over m in order
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int k = 0; k < 40; ++k) red[k][t] = acc[40 * h + k];
    __syncthreads();
    for (int o = t; o < 160; o += 256) {
      const int k = o >> 2, qq = o & 3;
      float sum = 0.0f;
      for (int m = 0; m < 64; ++m) sum += red[k][4 * m + qq];
      fin[qq * 80 + 40 * h + k] = sum;
    }
    __syncthreads();
  }
  float* out = part + int64_t(blockIdx.x) * 320;
  for (int j = t; j < 320; j += 256) {
    const int n = j < 288 ? j / 9 : j - 288;
    const float val = j < 288 ? fin[(n >> 3) * 80 + (n & 7) * 9 + (j - 9 * n)]
                              : fin[(n >> 3) * 80 + 72 + (n & 7)];
    __builtin_nontemporal_store(val, &out[j]);
  }
}

// Max-pooling backward fused with the skip addition and the ReLU mask:
// din[q] = (dout of q's window if q is the window's first maximal position,
// else 0) + skip[q], zeroed where in[q] <= 0 (bfloat16 out).  A thread takes
// one pooled pixel and 8 channels (16-byte loads and stores).
__global__ __launch_bounds__(256) void k_pool_bwd_add(const uint16_t* __restrict__ in, int B,
                                                      int H, int W, int C,
                                                      const uint16_t* __restrict__ dout,
                                                      const uint16_t* __restrict__ skip,
                                                      uint16_t* __restrict__ din) {
  const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
  // B * H * W <= 2^26 and C <= 256 (the network's shapes): 32-bit indices
  const int n = B * Ho * Wo * C8;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const int p = i / C8, c8 = i - p * C8;
    const int q = p / Wo, x = p - q * Wo, b = q / Ho, y = q - b * Ho;
    const int64_t base = ((int64_t(b) * H + 2 * y) * W + 2 * x) * C + 8 * c8;
    const int64_t off[4] = {0, C, int64_t(W) * C, int64_t(W) * C + C};
    uint4 v[4], sk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] = *reinterpret_cast<const uint4*>(in + base + off[q]);
      sk[q] = *reinterpret_cast<const uint4*>(skip + base + off[q]);
    }
    const uint4 dv = *reinterpret_cast<const uint4*>(dout + int64_t(p) * C + 8 * c8);
    const uint16_t* vh[4] = {reinterpret_cast<const uint16_t*>(&v[0]),
                             reinterpret_cast<const uint16_t*>(&v[1]),
                             reinterpret_cast<const uint16_t*>(&v[2]),
                             reinterpret_cast<const uint16_t*>(&v[3])};
    const uint16_t* dh = reinterpret_cast<const uint16_t*>(&dv);
    uint4 o[4];
    uint16_t* oh[4] = {reinterpret_cast<uint16_t*>(&o[0]), reinterpret_cast<uint16_t*>(&o[1]),
                       reinterpret_cast<uint16_t*>(&o[2]), reinterpret_cast<uint16_t*>(&o[3])};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int best = 0;
      float m = bf2f(vh[0][e]);
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        const float w = bf2f(vh[q][e]);
        if (w > m) {
          m = w;
          best = q;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float r = (q == best ? bf2f(dh[e]) : 0.0f) +
                  bf2f(reinterpret_cast<const uint16_t*>(&sk[q])[e]);
        if (!(bf2f(vh[q][e]) > 0.0f)) r = 0.0f;
        oh[q][e] = f2bf(r);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<uint4*>(din + base + off[q]) = o[q];
  }
}

// The output layer (1x1 convolution to one channel of a 32-channel input):
// y[p] = b + sum over c of w[c] * h[p][c], the products of bfloat16 values
// summed in FP32 in order of c.
__global__ __launch_bounds__(256) void k_out1_fwd(const uint16_t* __restrict__ h,
                                                  const uint16_t* __restrict__ w,
                                                  const float* __restrict__ bias, int64_t P,
                                                  float* __restrict__ y) {
  for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < P; p += int64_t(gridDim.x) * 256) {
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 v = *reinterpret_cast<const uint4*>(h + p * 32 + 8 * q);
      const uint16_t* vh = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int e = 0; e < 8; ++e) s = __builtin_fmaf(bf2f(w[8 * q + e]), bf2f(vh[e]), s);
    }
    y[p] = s + bias[0];
  }
}

// Squared-error loss and the output layer's backward pass in one sweep over
// the pixels: z = y[p] + res[p] (res nullable), d = z - t[p]; loss += sum of
// d^2 / P; the output gradient g = bf16(2 d / P); the input gradient
// gin[p][c] = bf16(g * w[c]) where h[p][c] > 0 (h: the layer input, a ReLU
// output), else 0; and the work-group's partial sums of g * h[p][c] (weight
// gradient, c < 32) and of g (bias gradient) into part[blockIdx.x][0 .. 35]
// (slots 33 .. 35 zero), summed over the work-group in a fixed order.
__global__ __launch_bounds__(256) void k_out1_bwd(const float* __restrict__ y,
                                                  const float* __restrict__ res,
                                                  const float* __restrict__ t, int64_t P,
                                                  const uint16_t* __restrict__ h,
                                                  const uint16_t* __restrict__ w,
                                                  uint16_t* __restrict__ gin,
                                                  float* __restrict__ loss,
                                                  float* __restrict__ part) {
  __shared__ float red[34][256];
  const float inv = 1.0f / float(P);
  float acc[33], ls = 0.0f;
#pragma unroll
  for (int c = 0; c < 33; ++c) acc[c] = 0.0f;
  float wf[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) wf[c] = bf2f(w[c]);
  for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < P; p += int64_t(gridDim.x) * 256) {
    const float d = (res ? y[p] + res[p] : y[p]) - t[p];
    ls += d * d;
    const float g = bf2f(f2bf(2.0f * d * inv));
    acc[32] += g;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 v = *reinterpret_cast<const uint4*>(h + p * 32 + 8 * q);
      const uint16_t* vh = reinterpret_cast<const uint16_t*>(&v);
      uint4 o;
      uint16_t* oh = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float hv = bf2f(vh[e]);
        acc[8 * q + e] = __builtin_fmaf(g, hv, acc[8 * q + e]);
        oh[e] = hv > 0.0f ? f2bf(g * wf[8 * q + e]) : uint16_t(0);
      }
      *reinterpret_cast<uint4*>(gin + p * 32 + 8 * q) = o;
    }
  }
  const int tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 33; ++c) red[c][tid] = acc[c];
  red[33][tid] = ls;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o)
      for (int c = 0; c < 34; ++c) red[c][tid] += red[c][tid + o];
    __syncthreads();
  }
  if (tid < 36) part[int64_t(blockIdx.x) * 36 + tid] = tid < 33 ? red[tid][0] : 0.0f;
  if (tid == 0 && loss) atomicAdd(loss, red[33][0] * inv);
}

__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, int C,
                                             const float* __restrict__ res,
                                             const float* __restrict__ t, int64_t P,
                                             float* __restrict__ loss, uint16_t* __restrict__ dy) {
  float s = 0.0f;
  const float inv = 1.0f / float(P);
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < P * C;
       i += int64_t(gridDim.x) * 256) {
    const int64_t p = i / C;
    const int c = int(i % C);
    float g = 0.0f;
    if (c == 0) {
      const float d = (res ? y[i] + res[p] : y[i]) - t[p];
      s += d * d;
      g = 2.0f * d * inv;
    }
    if (dy) dy[i] = f2bf(g);
  }
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] * inv);
}

// Adam on FP32 master parameters (bias-corrected moments).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Planes [B][H*W] (FP32) -> x = (p - mu) / sigma with the plane's own mean
// and population standard deviation (sigma = 1 for a constant plane), in two
// kernels.  k_norm_partial: work-group (b, s) sums slice s of plane b (FP64
// sum and sum of squares) into part[(b * S + s) * 2 + {0, 1}].
// k_norm_apply: every thread adds the S partials of its plane in slice order
// (the same result for every thread of the plane) and writes x as FP32 [B][H*W]
// in xf and as BF16 channel 0 of [B][H*W][C] (channels 1..C-1 zero); the
// plane's first thread writes stats[2b], stats[2b+1] = mu, sigma.  Targets, if
// given, take their plane's input transform (FP32, tnorm).
constexpr int kNormSlices = 16;

__global__ __launch_bounds__(256) void k_norm_partial(const float* __restrict__ planes,
                                                      int64_t hw, double* __restrict__ part) {
  const int b = blockIdx.x, sl = blockIdx.y;
  const int64_t per = (hw + kNormSlices - 1) / kNormSlices;
  const int64_t lo = sl * per, hi = lo + per < hw ? lo + per : hw;
  const float* p = planes + int64_t(b) * hw;
  double s = 0.0, s2 = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double v = p[i];
    s += v;
    s2 += v * v;
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[(int64_t(b) * kNormSlices + sl) * 2] = red[0][0];
    part[(int64_t(b) * kNormSlices + sl) * 2 + 1] = red[1][0];
  }
}

__global__ __launch_bounds__(256) void k_norm_apply(const float* __restrict__ planes, int B,
                                                    int64_t hw, int C,
                                                    const double* __restrict__ part,
                                                    uint16_t* __restrict__ out,
                                                    float* __restrict__ xf,
                                                    const float* __restrict__ targets,
                                                    float* __restrict__ tnorm,
                                                    float* __restrict__ stats) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < int64_t(B) * hw;
       i += int64_t(gridDim.x) * 256) {
    const int b = int(i / hw);
    double s = 0.0, s2 = 0.0;
    for (int k = 0; k < kNormSlices; ++k) {
      s += part[(int64_t(b) * kNormSlices + k) * 2];
      s2 += part[(int64_t(b) * kNormSlices + k) * 2 + 1];
    }
    const double mean = s / double(hw);
    const double var = s2 / double(hw) - mean * mean;
    const float sd = float(var > 0.0 ? sqrt(var) : 1.0);
    const float mu = float(mean);
    if (i % hw == 0 && stats) {
      stats[2 * b] = mu;
      stats[2 * b + 1] = sd;
    }
    const float x = (planes[i] - mu) / sd;
    xf[i] = x;
    if (C == 8) {
      *reinterpret_cast<uint4*>(out + i * 8) = make_uint4(f2bf(x), 0u, 0u, 0u);
    } else {
      out[i * C] = f2bf(x);
      for (int c = 1; c < C; ++c) out[i * C + c] = 0;
    }
    if (targets) tnorm[i] = (targets[i] - mu) / sd;
  }
}

// y[b][i] = (x[b][i][0] + res[b][i]) * sigma_b + mu_b (back to the plane's
// own scale)
__global__ __launch_bounds__(256) void k_denormalize(const float* __restrict__ x, int C,
                                                     const float* __restrict__ res,
                                                     const float* __restrict__ stats, int64_t hw,
                                                     int B, float* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < int64_t(B) * hw;
       i += int64_t(gridDim.x) * 256) {
    const int b = int(i / hw);
    y[i] = (x[i * C] + res[i]) * stats[2 * b + 1] + stats[2 * b];
  }
}

// ---- image quality -------------------------------------------------------------
// One work-group per plane, FP64: PSNR with the target's data range
// max(t) - min(t) (infinite when the planes are equal), and SSIM with an
// 11 x 11 Gaussian window (sigma 1.5, normalised to sum 1) over every position
// where the window fits, both planes mapped to [0, 1] by the target's minimum
// and range (range 1 for a constant target), K1 = 0.01, K2 = 0.03.
__global__ __launch_bounds__(256) void k_quality(const float* __restrict__ pred,
                                                 const float* __restrict__ target, int H, int W,
                                                 double* __restrict__ psnr,
                                                 double* __restrict__ ssim) {
  const int b = blockIdx.x;
  const int64_t hw = int64_t(H) * W;
  const float* p = pred + int64_t(b) * hw;
  const float* t = target + int64_t(b) * hw;
  __shared__ double red[3][256];
  __shared__ double win[11];
  double lo = __builtin_huge_val(), hi = -__builtin_huge_val(), se = 0.0;
  for (int64_t i = threadIdx.x; i < hw; i += 256) {
    const double tv = t[i];
    lo = fmin(lo, tv);
    hi = fmax(hi, tv);
    const double d = double(p[i]) - tv;
    se += d * d;
  }
  red[0][threadIdx.x] = lo;
  red[1][threadIdx.x] = hi;
  red[2][threadIdx.x] = se;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) {
      red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + o]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + o]);
      red[2][threadIdx.x] += red[2][threadIdx.x + o];
    }
    __syncthreads();
  }
  lo = red[0][0];
  const double range = red[1][0] - lo;
  se = red[2][0];
  if (threadIdx.x == 0) {
    psnr[b] = se == 0.0 ? __builtin_huge_val()
                        : 10.0 * log10(range * range / (se / double(hw)));
    double g[11], sum = 0.0;
    for (int i = 0; i < 11; ++i) {
      const double r = double(i - 5);
      g[i] = exp(-(r * r) / (2.0 * 1.5 * 1.5));
      sum += g[i];
    }
    for (int i = 0; i < 11; ++i) win[i] = g[i] / sum;   // 2-D window = win x win
  }
  __syncthreads();
  const double inv = 1.0 / (range == 0.0 ? 1.0 : range);
  const double c1 = 0.01 * 0.01, c2 = 0.03 * 0.03;
  const int ny = H - 10, nx = W - 10;
  double acc = 0.0;
  for (int64_t q = threadIdx.x; q < int64_t(ny) * nx; q += 256) {
    const int y0 = int(q / nx), x0 = int(q % nx);
    double sa = 0, sb = 0, saa = 0, sbb = 0, sab = 0;
    for (int i = 0; i < 11; ++i) {
      for (int j = 0; j < 11; ++j) {
        const double w = win[i] * win[j];
        const int64_t o = int64_t(y0 + i) * W + x0 + j;
        const double a = (double(p[o]) - lo) * inv;
        const double c = (double(t[o]) - lo) * inv;
        sa += w * a;
        sb += w * c;
        saa += w * a * a;
        sbb += w * c * c;
        sab += w * a * c;
      }
    }
    const double va = saa - sa * sa, vb = sbb - sb * sb, cab = sab - sa * sb;
    acc += ((2.0 * sa * sb + c1) * (2.0 * cab + c2)) /
           ((sa * sa + sb * sb + c1) * (va + vb + c2));
  }
  __syncthreads();
  red[2][threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[2][threadIdx.x] += red[2][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) ssim[b] = red[2][0] / double(int64_t(ny) * nx);
}

}  // namespace

template <int KS, int TM, int TN>
void launch_conv(const NnConvArgs& a, hipStream_t s) {
  const int64_t M = int64_t(a.B) * a.H * a.W;
  hipLaunchKernelGGL((k_conv<KS, TM, TN>), dim3(unsigned((M + 64 * TM - 1) / (64 * TM)),
                                                unsigned(a.Cout / (16 * TN))),
                     dim3(256), 0, s, a);
}

template <int KS>
void conv_ks(const NnConvArgs& a, hipStream_t s) {
  // the largest tile whose grid still holds ~2 work-groups per compute unit
  const int64_t M = int64_t(a.B) * a.H * a.W;
  auto groups = [&](int tm, int tn) { return ((M + 64 * tm - 1) / (64 * tm)) * (a.Cout / (16 * tn)); };
  constexpr int64_t kMin = 512;
  if (a.Cout % 64 == 0 && groups(4, 4) >= kMin)
    launch_conv<KS, 4, 4>(a, s);
  else if (a.Cout % 64 == 0 && groups(2, 4) >= kMin)
    launch_conv<KS, 2, 4>(a, s);
  else if (groups(4, 2) >= kMin)
    launch_conv<KS, 4, 2>(a, s);
  else if (groups(2, 2) >= kMin)
    launch_conv<KS, 2, 2>(a, s);
  else
    launch_conv<KS, 1, 2>(a, s);
}

// Kernel rows per phase: all three (one phase per chunk of 32 input
// channels) for 64-channel tiles; one for 128-channel tiles, whose nine
// taps' weights would not leave room for a second work-group, and for
// 32-channel tiles, whose level-0 grids gain more from occupancy.
template <int TM, int TN, int WM, int WN>
void launch_conv3_lds(const NnConvArgs& a, hipStream_t s) {
  constexpr int TH = WM * TM, NT = WN * TN * 16;
  constexpr int KY = NT == 64 ? 3 : 1;
  const int64_t blocks = int64_t((a.W + 15) / 16) * ((a.H + TH - 1) / TH) * a.B;
  const dim3 grid(unsigned(blocks), unsigned(a.Cout / NT));
  if constexpr (TM % 2 == 0) {
    if (a.dlow) {
      hipLaunchKernelGGL((k_conv3_lds<TM, TN, WM, WN, KY, 2>), grid, dim3(256), 0, s, a);
      return;
    }
  }
  if (a.pool_in)
    hipLaunchKernelGGL((k_conv3_lds<TM, TN, WM, WN, KY, 1>), grid, dim3(256), 0, s, a);
  else if (a.low)
    hipLaunchKernelGGL((k_conv3_lds<TM, TN, WM, WN, KY, 3>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_conv3_lds<TM, TN, WM, WN, KY, 0>), grid, dim3(256), 0, s, a);
}

// Work-groups of the LDS-staged 3x3 kernel for a tile of TH rows and NT channels.
int64_t lds_groups(const NnConvArgs& a, int th, int nt) {
  return int64_t((a.W + 15) / 16) * ((a.H + th - 1) / th) * a.B * (a.Cout / nt);
}

// The LDS-staged tile for a 3x3 layer with Cin % 32 == 0: the first shape
// (rows x channels: 8 x 128, 8 x 64, 4 x 64, 16 x 32, 8 x 32, 4 x 32) whose
// grid holds >= 512 work-groups, failing that >= 256, then >= 128; -1: none
// (the register-fed kernel).
int conv3_tile(const NnConvArgs& a) {
  if (a.ks != 3 || a.Cin % 32 != 0) return -1;
  for (int64_t kMin = 512; kMin >= 128; kMin /= 2) {
    if (a.Cout % 128 == 0 && lds_groups(a, 8, 128) >= kMin) return 0;
    if (a.Cout % 64 == 0 && lds_groups(a, 8, 64) >= kMin) return 1;
    if (a.Cout % 64 == 0 && lds_groups(a, 4, 64) >= kMin) return 2;
    if (lds_groups(a, 16, 32) >= kMin) return 3;
    if (lds_groups(a, 8, 32) >= kMin) return 4;
    if (lds_groups(a, 4, 32) >= kMin) return 5;
  }
  return -1;
}

bool nn_conv_takes_split(const NnConvArgs& a) {
  if (a.low || a.pool_in || a.out || a.out_f32 || a.bias || a.relu || a.mask) return false;
  if (a.H % 2 || a.W % 2 || a.c1 <= 0 || a.c1 >= a.Cout) return false;
  // tiles 0 .. 4 have an even number of rows per wave; tile channel widths
  // 128, 64, 64, 32, 32 must divide c1
  const int tile = conv3_tile(a);
  static const int nt[5] = {128, 64, 64, 32, 32};
  return tile >= 0 && tile <= 4 && a.c1 % nt[tile] == 0 && (a.Cout - a.c1) % 8 == 0;
}

bool nn_conv_takes_low(const NnConvArgs& a) {
  if (a.low && a.pool_in) return false;
  if (a.low && (a.c_low % 32 || a.H % 2 || a.W % 2)) return false;
  return conv3_tile(a) >= 0;
}

hipError_t nn_conv(const NnConvArgs& a, hipStream_t s) {
  if ((a.low || a.pool_in) && !nn_conv_takes_low(a)) return hipErrorInvalidValue;
  if ((a.dlow || a.dskip) && (!a.dlow || !a.dskip || !nn_conv_takes_split(a))) return hipErrorInvalidValue;
  const int tile = conv3_tile(a);
  if (tile >= 0) {
    switch (tile) {
      case 0: launch_conv3_lds<4, 4, 2, 2>(a, s); break;
      case 1: launch_conv3_lds<4, 2, 2, 2>(a, s); break;
      case 2: launch_conv3_lds<2, 2, 2, 2>(a, s); break;
      case 3: launch_conv3_lds<4, 2, 4, 1>(a, s); break;
      case 4: launch_conv3_lds<2, 2, 4, 1>(a, s); break;
      default: launch_conv3_lds<1, 2, 4, 1>(a, s); break;
    }
  } else if (a.ks == 3) {
    conv_ks<3>(a, s);
  } else if (a.ks == 1) {
    conv_ks<1>(a, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Launch shape of a weight gradient: the kernel (3x3 all-taps kernel with
// NT = 64 or 32 and block width TW = 64, 32 or 16; else the general kernel
// for ks = 3 or 1 with NT = 64 or 32) and the grid, whose z dimension splits
// the pixels.
struct WgradPlan {
  int kind;  // 0..5: k_conv3_wgrad (NT 64: TW 64, 32, 16; NT 32: TW 64, 32, 16); 6..9: k_conv_wgrad
  unsigned gx, gy, gz;
};

WgradPlan wgrad_plan(const NnWgradArgs& a) {
  WgradPlan p{};
  const bool wide = a.Cout % 64 == 0;
  const int NT = wide ? 64 : 32;
  p.gx = unsigned(a.Cout / NT);
  int64_t z;
  if (a.ks == 3 && a.Cin % 32 == 0) {
    const int tw = a.W >= 64 ? 64 : a.W >= 32 ? 32 : 16;
    const int rows = (wide ? 128 : 256) / tw;
    p.kind = (wide ? 0 : 3) + (tw == 64 ? 0 : tw == 32 ? 1 : 2);
    p.gy = unsigned(a.Cin / 32);
    const int64_t nb = int64_t(a.B) * ((a.H + rows - 1) / rows) * ((a.W + tw - 1) / tw);
    // up to ~256 work-groups (one per compute unit), each of >= 2 blocks
    z = 256 / (int64_t(p.gx) * p.gy);
    if (z > nb / 2) z = nb / 2;
  } else {
    p.kind = 6 + (a.ks == 1 ? 2 : 0) + (wide ? 0 : 1);
    p.gy = unsigned((a.Kpad + 63) / 64);
    const int64_t M = int64_t(a.B) * a.H * a.W;
    // up to ~2048 work-groups, each of >= 512 pixels
    z = 2048 / (int64_t(p.gx) * p.gy);
    if (z > M / 512) z = M / 512;
  }
  if (z < 1) z = 1;
  if (z > 65535) z = 65535;
  p.gz = unsigned(z);
  return p;
}

int64_t nn_conv_wgrad_part_floats(const NnWgradArgs& a) {
  const WgradPlan p = wgrad_plan(a);
  return int64_t(p.gz) * (int64_t(a.Cout) * a.ks * a.ks * a.Cin + a.Cout);
}

hipError_t nn_conv_wgrad(const NnWgradArgs& a, hipStream_t s, int phases) {
  if (a.ks != 3 && a.ks != 1) return hipErrorInvalidValue;
  if ((phases & 2) && !(phases & 1) && !a.part) return hipErrorInvalidValue;
  const WgradPlan p = wgrad_plan(a);
  if ((a.low || a.pool_in) &&
      (p.kind > 5 || (a.low && a.pool_in) || (a.low && (a.c_low % 32 || a.H % 2 || a.W % 2))))
    return hipErrorInvalidValue;
  if (a.part && a.part_cap < nn_conv_wgrad_part_floats(a)) return hipErrorInvalidValue;
  const dim3 grid(p.gx, p.gy, p.gz), block(256);
  if (phases & 1) switch (p.kind) {
    case 0: hipLaunchKernelGGL((k_conv3_wgrad<64, 64, 2>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_conv3_wgrad<64, 32, 4>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_conv3_wgrad<64, 16, 8>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_conv3_wgrad<32, 64, 4>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_conv3_wgrad<32, 32, 8>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_conv3_wgrad<32, 16, 16>), grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_conv_wgrad<3, 64, 64>), grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_conv_wgrad<3, 32, 64>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_conv_wgrad<1, 64, 64>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((k_conv_wgrad<1, 32, 64>), grid, block, 0, s, a); break;
  }
  if (a.part && (phases & 2)) {
    const int64_t nw = int64_t(a.Cout) * a.ks * a.ks * a.Cin;
    int64_t blocks = (nw + a.Cout + 63) / 64;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(unsigned(blocks)), dim3(256), 0, s, a.part,
                       int(p.gz), nw, a.Cout, a.dw, a.db);
  }
  return hipGetLastError();
}

hipError_t nn_bias_grad(const uint16_t* dy, int64_t M, int C, float* db, hipStream_t s) {
  int64_t gx = (M + 3) / 4;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(k_bias_grad, dim3(unsigned(gx), unsigned((C + 63) / 64)), dim3(256), 0, s, dy,
                     M, C, db);
  return hipGetLastError();
}

hipError_t nn_pack_weights(const float* w, int Cout, int Cin, int ks, uint16_t* wf, int kpad,
                           uint16_t* wt, int kpad_t, hipStream_t s) {
  const int64_t n = int64_t(Cout) * kpad + (wt ? int64_t(Cin) * kpad_t : 0);
  hipLaunchKernelGGL(k_pack_weights, dim3(grid1(n)), dim3(256), 0, s, w, Cout, Cin, ks, wf, kpad,
                     wt, kpad_t);
  return hipGetLastError();
}

hipError_t nn_maxpool(const uint16_t* in, int B, int H, int W, int C, uint16_t* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_maxpool, dim3(grid1(int64_t(B) * (H / 2) * (W / 2) * C)), dim3(256), 0, s,
                     in, B, H, W, C, out);
  return hipGetLastError();
}

hipError_t nn_maxpool_bwd(const uint16_t* in, int B, int H, int W, int C, const uint16_t* dout,
                          uint16_t* din, hipStream_t s) {
  hipLaunchKernelGGL(k_maxpool_bwd, dim3(grid1(int64_t(B) * (H / 2) * (W / 2) * C)), dim3(256), 0,
                     s, in, B, H, W, C, dout, din);
  return hipGetLastError();
}

hipError_t nn_upsample(const uint16_t* in, int B, int H, int W, int C, uint16_t* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_upsample, dim3(grid1(int64_t(B) * 4 * H * W * C)), dim3(256), 0, s, in, B, H,
                     W, C, out);
  return hipGetLastError();
}

hipError_t nn_upsample_bwd(const uint16_t* dout, int B, int H, int W, int C, const uint16_t* mask,
                           uint16_t* din, hipStream_t s) {
  hipLaunchKernelGGL(k_upsample_bwd, dim3(grid1(int64_t(B) * H * W * C)), dim3(256), 0, s, dout, B,
                     H, W, C, mask, din);
  return hipGetLastError();
}

hipError_t nn_concat(const uint16_t* a, const uint16_t* b, int64_t P, int C1, int C2, uint16_t* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_concat, dim3(grid1(P * (C1 + C2))), dim3(256), 0, s, a, b, P, C1, C2, out, 0);
  return hipGetLastError();
}

hipError_t nn_split(const uint16_t* d, int64_t P, int C1, int C2, uint16_t* da, uint16_t* db,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_concat, dim3(grid1(P * (C1 + C2))), dim3(256), 0, s, da, db, P, C1, C2,
                     const_cast<uint16_t*>(d), 1);
  return hipGetLastError();
}

hipError_t nn_upcat(const uint16_t* low, const uint16_t* skip, int B, int H, int W, int C1, int C2,
                    uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_upcat, dim3(grid1(int64_t(B) * 4 * H * W * ((C1 + C2) / 8))), dim3(256), 0,
                     s, low, skip, B, H, W, C1, C2, out);
  return hipGetLastError();
}

hipError_t nn_upcat_grad(const uint16_t* d, int B, int H, int W, int C1, int C2,
                         const uint16_t* mask, uint16_t* dlow, uint16_t* dskip, hipStream_t s) {
  const int64_t n = int64_t(B) * H * W * (C1 / 8) + int64_t(B) * 4 * H * W * (C2 / 8);
  hipLaunchKernelGGL(k_upcat_grad, dim3(grid1(n)), dim3(256), 0, s, d, B, H, W, C1, C2, mask, dlow,
                     dskip);
  return hipGetLastError();
}

hipError_t nn_add_mask(uint16_t* x, const uint16_t* add, const uint16_t* mask, int64_t n,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_add_mask, dim3(grid1(n)), dim3(256), 0, s, x, add, mask, n);
  return hipGetLastError();
}

hipError_t nn_mse(const float* y, int C, const float* res, const float* t, int64_t P, float* loss,
                  uint16_t* dy, hipStream_t s) {
  int64_t g = (P * C + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_mse, dim3(unsigned(g)), dim3(256), 0, s, y, C, res, t, P, loss, dy);
  return hipGetLastError();
}

hipError_t nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                   float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

size_t nn_normalize_scratch_bytes(int B) { return size_t(B) * kNormSlices * 2 * sizeof(double); }

hipError_t nn_normalize(const float* planes, int B, int64_t hw, int C, uint16_t* out, float* xf,
                        const float* targets, float* tnorm, float* stats, double* scratch,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_norm_partial, dim3(unsigned(B), unsigned(kNormSlices)), dim3(256), 0, s,
                     planes, hw, scratch);
  hipLaunchKernelGGL(k_norm_apply, dim3(grid1(int64_t(B) * hw)), dim3(256), 0, s, planes, B, hw, C,
                     scratch, out, xf, targets, tnorm, stats);
  return hipGetLastError();
}

hipError_t nn_pack_all(const float* params, uint16_t* packed, const NnPackTable& tab,
                       hipStream_t s) {
  int64_t most = 0;
  for (int l = 0; l < tab.n; ++l) {
    const NnPackLayer& L = tab.layer[l];
    const int64_t n = int64_t(L.cout) * L.kpad + (L.transposed ? int64_t(L.cin) * L.kpad_t : 0);
    if (n > most) most = n;
  }
  if (most >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  int64_t gx = (most + 4 * 256 - 1) / (4 * 256);  // about four elements per thread
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(k_pack_all, dim3(unsigned(gx), unsigned(tab.n)), dim3(256), 0, s, params,
                     packed, tab);
  return hipGetLastError();
}

hipError_t nn_denormalize(const float* x, int C, const float* res, const float* stats, int64_t hw,
                          int B, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_denormalize, dim3(grid1(int64_t(B) * hw)), dim3(256), 0, s, x, C, res, stats,
                     hw, B, y);
  return hipGetLastError();
}

hipError_t nn_in1_fwd(const uint16_t* x, int B, int H, int W, int cx, const uint16_t* wk, int kpad,
                      const float* bias, uint16_t* out, hipStream_t s) {
  if (int64_t(B) * H * W >= (int64_t(1) << 30)) return hipErrorInvalidValue;  // 32-bit indices
  hipLaunchKernelGGL(k_in1_fwd, dim3(grid1((int64_t(B) * H * W + 1) / 2)), dim3(256), 0, s, x, B,
                     H, W, cx, wk, kpad, bias, out);
  return hipGetLastError();
}

int nn_in1_wgrad_groups(int64_t P) {
  int64_t g = (P + 511) / 512;  // about eight pixels per thread
  if (g < 1) g = 1;
  if (g > 512) g = 512;
  return int(g);
}

hipError_t nn_in1_wgrad(const uint16_t* x, int B, int H, int W, int cx, const uint16_t* dy,
                        float* part, float* dw, float* db, hipStream_t s, int phases) {
  if (int64_t(B) * H * W >= (int64_t(1) << 30)) return hipErrorInvalidValue;  // 32-bit indices
  const int g = nn_in1_wgrad_groups(int64_t(B) * H * W);
  if (phases & 1)
    hipLaunchKernelGGL(k_in1_wgrad, dim3(unsigned(g)), dim3(256), 0, s, x, B, H, W, cx, dy, part);
  if (phases & 2)
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(5), dim3(256), 0, s, part, g, int64_t(288), 32, dw, db,
                       cx);
  return hipGetLastError();
}

hipError_t nn_pool_bwd_add(const uint16_t* in, int B, int H, int W, int C, const uint16_t* dout,
                           const uint16_t* skip, uint16_t* din, hipStream_t s) {
  if (int64_t(B) * H * W * C >= (int64_t(1) << 31)) return hipErrorInvalidValue;  // 32-bit indices
  hipLaunchKernelGGL(k_pool_bwd_add, dim3(grid1(int64_t(B) * (H / 2) * (W / 2) * (C / 8))),
                     dim3(256), 0, s, in, B, H, W, C, dout, skip, din);
  return hipGetLastError();
}

hipError_t nn_out1_fwd(const uint16_t* h, const uint16_t* w, const float* bias, int64_t P, float* y,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_out1_fwd, dim3(grid1(P)), dim3(256), 0, s, h, w, bias, P, y);
  return hipGetLastError();
}

int nn_out1_bwd_groups(int64_t P) {
  int64_t g = (P + 1023) / 1024;  // about four pixels per thread
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  return int(g);
}

hipError_t nn_out1_bwd(const float* y, const float* res, const float* t, int64_t P,
                       const uint16_t* h, const uint16_t* w, uint16_t* gin, float* loss,
                       float* part, float* dw, float* db, hipStream_t s) {
  const int g = nn_out1_bwd_groups(P);
  hipLaunchKernelGGL(k_out1_bwd, dim3(unsigned(g)), dim3(256), 0, s, y, res, t, P, h, w, gin, loss,
                     part);
  // rows of 36: 32 weight slots, then db[0 .. 3] (slots 1 .. 3 add zero)
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(1), dim3(256), 0, s, part, g, int64_t(32), 4, dw, db);
  return hipGetLastError();
}

hipError_t nn_quality(const float* pred, const float* target, int B, int H, int W, double* psnr,
                      double* ssim, hipStream_t s) {
  hipLaunchKernelGGL(k_quality, dim3(unsigned(B)), dim3(256), 0, s, pred, target, H, W, psnr, ssim);
  return hipGetLastError();
}

}  // namespace cpi
