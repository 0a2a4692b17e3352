// Sum of products S_ab = A^T B on int8 matrix cores (v_mfma_i32_16x16x64_i8),
// followed by the exact combination of Eq. (1):
//     numer = N * S_ab - S_a * S_b        (int64)
//     gamma = fl64(fl64(numer) / fl64(N * N))
//     gamma_f32 = fl32(gamma)
//
// Operands are pixel-major rows (frames contiguous) built by the ingest
// kernels.  M = detector-B pixels (views), N = detector-A pixels, so the
// matrix-core output rows are views and its columns run along detector-A
// pixels, which is the view-major storage of Gamma.
//
// Each 64-byte segment of a row holds 512 frames as bits or 64 frames as
// bytes.  Lane l of a wave reads 16 bytes of row (16*f + l%16) at byte
// 16*(l/16) of the segment.  For byte rows those 16 bytes are the lane's
// 16 K values of one MFMA.  For bit rows they are four 32-bit words; word w
// shifted right by s and masked with 0x01010101 gives four bytes holding the
// frames 8*b + s of that word (b = 0..3), so shifts 4h..4h+3 make one 16-byte
// MFMA operand and every word feeds two MFMAs.  Both operands use the same
// lane/byte -> frame assignment, so every product pairs A and B of the same
// frame, whatever order the hardware sums the K index in.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include "kernels.h"

namespace cpi {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Work-group b executes on XCD b % 8.  Give each XCD a contiguous range of
// output tiles so that tiles sharing operand rows share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
  const int per = nwg >> 3, rem = nwg & 7;
  const int x = b & 7, i = b >> 3;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + i;
}

// Epilogue fields, copied out of the kernel argument block into registers.
struct Epi {
  int mode, layout;
  int64_t pa, pb, n, kchunk;
  const int64_t* sum_a;
  const int64_t* sum_b;
  const int64_t* csum_a;
  const int64_t* csum_b;
  double* gamma;
  float* gamma_f32;
  int64_t* numer;
  int64_t* acc64;
  int32_t* acc32;
};

template <int MODE>
__device__ __forceinline__ void store_result(const Epi& g, int64_t q, int64_t p, int64_t s,
                                             int64_t o) {
  // s: sum of products in the operand domain; o: operand offset (0 or 128)
  const int64_t idx_vm = q * g.pa + p;
  const int64_t n = g.n;
  switch (MODE) {
    case EPI_STORE64:
      g.acc64[idx_vm] = s;
      return;
    case EPI_ADD64:
      g.acc64[idx_vm] += s;
      return;
    case EPI_FINAL_ACC64:
      s += g.acc64[idx_vm];
      break;
    case EPI_STREAM32: {
      const int32_t t = g.acc32[idx_vm] + int32_t(s);
      g.acc32[idx_vm] = t;
      s = t;
      o = 0;
      break;
    }
    case EPI_STREAM64: {
      // back to raw values: sum (a-o)(b-o) = S_ab - o S_a - o S_b + k o^2
      const int64_t raw = s + o * (g.csum_a[p] + g.csum_b[q]) - g.kchunk * o * o;
      const int64_t t = g.acc64[idx_vm] + raw;
      g.acc64[idx_vm] = t;
      s = t;
      o = 0;
      break;
    }
    default:
      break;
  }
  const int64_t sa = g.sum_a[p] - o * n;
  const int64_t sb = g.sum_b[q] - o * n;
  const int64_t numer = n * s - sa * sb;
  const double nn = double(n) * double(n);
  const double gam = double(numer) / nn;
  const int64_t idx = (g.layout == CPI_GAMMA_VIEW_MAJOR) ? idx_vm : p * g.pb + q;
  if (g.gamma) g.gamma[idx] = gam;
  if (g.gamma_f32) g.gamma_f32[idx] = float(gam);
  if (g.numer) g.numer[idx] = numer;
}

template <int FM, int FN, bool BITS, int MODE, int SCHED, bool PF = true>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  if (g.cond) {
    const uint32_t mx = g.stats[0];
    if ((g.cond == 1) != (mx <= 1u)) return;
  }
  constexpr int WM = 16 * FM, WN = 16 * FN;
  const int tiles_m = int(g.m_pad / (2 * WM));
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int tm = id % tiles_m, tn = id / tiles_m;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, kg = lane >> 4;
  const int64_t m0 = int64_t(tm) * (2 * WM) + (wave & 1) * WM;
  const int64_t n0 = int64_t(tn) * (2 * WN) + (wave >> 1) * WN;
  const uint8_t* pm = g.opm + (m0 + r) * g.row_bytes + g.k_byte_off + kg * 16;
  const uint8_t* pn = g.opn + (n0 + r) * g.row_bytes + g.k_byte_off + kg * 16;
  const int64_t fstride = 16 * g.row_bytes;

  v4i acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4i{0, 0, 0, 0};

  v4i am[FM], bn[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) am[i] = *reinterpret_cast<const v4i*>(pm + i * fstride);
#pragma unroll
  for (int j = 0; j < FN; ++j) bn[j] = *reinterpret_cast<const v4i*>(pn + j * fstride);

  for (int64_t kb = 0; kb < g.kblocks; ++kb) {
    // next block's operands: loaded now (PF) or at the end of the iteration
    const int64_t nx = (kb + 1 < g.kblocks ? kb + 1 : kb) * 64;
    v4i am2[FM], bn2[FN];
    if constexpr (PF) {
#pragma unroll
      for (int i = 0; i < FM; ++i) am2[i] = *reinterpret_cast<const v4i*>(pm + i * fstride + nx);
#pragma unroll
      for (int j = 0; j < FN; ++j) bn2[j] = *reinterpret_cast<const v4i*>(pn + j * fstride + nx);
    }

    if constexpr (BITS) {
      const int mask = 0x01010101;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          v4i ea[FM], eb[FN];
#pragma unroll
          for (int i = 0; i < FM; ++i) {
            const uint32_t x = uint32_t(am[i][w]);
            ea[i] = v4i{int((x >> (4 * h + 0)) & mask), int((x >> (4 * h + 1)) & mask),
                        int((x >> (4 * h + 2)) & mask), int((x >> (4 * h + 3)) & mask)};
          }
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const uint32_t x = uint32_t(bn[j][w]);
            eb[j] = v4i{int((x >> (4 * h + 0)) & mask), int((x >> (4 * h + 1)) & mask),
                        int((x >> (4 * h + 2)) & mask), int((x >> (4 * h + 3)) & mask)};
          }
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ea[i], eb[j], acc[i][j], 0, 0, 0);
          if constexpr (SCHED > 0) {
            // one matrix-core op, then SCHED vector ops (the next step's bit
            // expansion), repeated over the step's FM*FN products
#pragma unroll
            for (int q = 0; q < FM * FN; ++q) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
              __builtin_amdgcn_sched_group_barrier(0x002, SCHED, 0);
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(am[i], bn[j], acc[i][j], 0, 0, 0);
    }
    if constexpr (!PF) {
#pragma unroll
      for (int i = 0; i < FM; ++i) am2[i] = *reinterpret_cast<const v4i*>(pm + i * fstride + nx);
#pragma unroll
      for (int j = 0; j < FN; ++j) bn2[j] = *reinterpret_cast<const v4i*>(pn + j * fstride + nx);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) am[i] = am2[i];
#pragma unroll
    for (int j = 0; j < FN; ++j) bn[j] = bn2[j];
  }

  int64_t o = 0;
  if (!BITS && g.offset_from_stats && g.stats[0] > 127u) o = 128;
  const Epi e{g.mode,   g.layout, g.pa,        g.pb,    g.n,     g.kchunk, g.sum_a, g.sum_b,
              g.csum_a, g.csum_b, g.gamma,     g.gamma_f32, g.numer, g.acc64,  g.acc32};
  // Output element (row 4*kg + t, column r) of each 16 x 16 tile.
#pragma clang loop unroll(full)
  for (int i = 0; i < FM; ++i)
#pragma clang loop unroll(full)
    for (int j = 0; j < FN; ++j)
#pragma clang loop unroll(full)
      for (int t = 0; t < 4; ++t) {
        const int64_t q = m0 + 16 * i + 4 * kg + t;
        const int64_t p = n0 + 16 * j + r;
        if (q < e.pb && p < e.pa) store_result<MODE>(e, q, p, int64_t(acc[i][j][t]), o);
      }
}

// One thread per Gamma element of a streaming state.
__global__ __launch_bounds__(256) void k_state_gamma(const void* __restrict__ sab, int sab64,
                                                     const int64_t* __restrict__ sum_a,
                                                     const int64_t* __restrict__ sum_b, int64_t n,
                                                     int64_t pa, int64_t pb, int layout,
                                                     double* __restrict__ gamma,
                                                     float* __restrict__ gamma_f32,
                                                     int64_t* __restrict__ numer) {
  const int64_t count = pa * pb;
  const double nn = double(n) * double(n);
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * 256) {
    const int64_t q = i / pa, p = i - q * pa;   // view-major element (q, p)
    const int64_t s = sab64 ? reinterpret_cast<const int64_t*>(sab)[i]
                            : int64_t(reinterpret_cast<const int32_t*>(sab)[i]);
    const int64_t num = n * s - sum_a[p] * sum_b[q];
    const double gam = double(num) / nn;
    const int64_t idx = (layout == CPI_GAMMA_VIEW_MAJOR) ? i : p * pb + q;
    if (gamma) gamma[idx] = gam;
    if (gamma_f32) gamma_f32[idx] = float(gam);
    if (numer) numer[idx] = num;
  }
}

struct TileChoice {
  int fm, fn, sched, pf;
};

// Contraction tile of the bit-row kernel: wave tile 16*fm x 16*fn, the
// interleave of bit expansion with matrix-core ops, register prefetch of the
// next operand block.  CPI_GEMM_TILE="FMxFN[sS][pP]" overrides the default
// (measurement runs).
TileChoice tile_choice() {
  static TileChoice t = [] {
    TileChoice c{4, 4, 0, 1};
    if (const char* v = std::getenv("CPI_GEMM_TILE")) {
      int fm = 0, fn = 0, sc = 0, pf = 1;
      if (std::sscanf(v, "%dx%ds%dp%d", &fm, &fn, &sc, &pf) >= 2) c = TileChoice{fm, fn, sc, pf};
    }
    return c;
  }();
  return t;
}

template <int FM, int FN, bool BITS, int MODE, int SCHED, bool PF = true>
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles_m = a.m_pad / (32 * FM);
  const int64_t tiles_n = a.n_pad / (32 * FN);
  if (tiles_m * (32 * FM) != a.m_pad || tiles_n * (32 * FN) != a.n_pad) return hipErrorInvalidValue;
  const int64_t nwg = tiles_m * tiles_n;
  if (nwg <= 0 || nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<FM, FN, BITS, MODE, SCHED, PF>), dim3(unsigned(nwg)), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_bits(const GemmArgs& a, hipStream_t s) {
  const TileChoice t = tile_choice();
  if (t.fm == 8 && t.fn == 4) return launch_gemm<8, 4, true, MODE, 0>(a, s);
  if (t.fm == 4 && t.fn == 4 && t.sched == 0 && t.pf == 0)
    return launch_gemm<4, 4, true, MODE, 0, false>(a, s);
  if (t.fm == 4 && t.fn == 4 && t.sched == 2) return launch_gemm<4, 4, true, MODE, 2>(a, s);
  if (t.fm == 2 && t.fn == 4) return launch_gemm<2, 4, true, MODE, 0>(a, s);
  if (t.fm == 4 && t.fn == 2) return launch_gemm<4, 2, true, MODE, 0>(a, s);
  return launch_gemm<4, 4, true, MODE, 0>(a, s);
}

}  // namespace

hipError_t gemm_correlate(const GemmArgs& a, bool bits, hipStream_t s) {
  switch (a.mode) {
    case EPI_FINAL:
      return bits ? launch_bits<EPI_FINAL>(a, s) : launch_gemm<4, 4, false, EPI_FINAL, 0>(a, s);
    case EPI_STREAM32:
      return bits ? launch_bits<EPI_STREAM32>(a, s)
                  : launch_gemm<4, 4, false, EPI_STREAM32, 0>(a, s);
    case EPI_FINAL_ACC64:
      return launch_gemm<4, 4, false, EPI_FINAL_ACC64, 0>(a, s);
    case EPI_STORE64:
      return launch_gemm<4, 4, false, EPI_STORE64, 0>(a, s);
    case EPI_ADD64:
      return launch_gemm<4, 4, false, EPI_ADD64, 0>(a, s);
    case EPI_STREAM64:
      return bits ? launch_gemm<4, 4, true, EPI_STREAM64, 0>(a, s)
                  : launch_gemm<4, 4, false, EPI_STREAM64, 0>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t state_gamma(const void* sab, bool sab64, const int64_t* sum_a, const int64_t* sum_b,
                       int64_t n, int64_t pa, int64_t pb, int layout, double* gamma,
                       float* gamma_f32, int64_t* numer, hipStream_t s) {
  int64_t gr = (pa * pb + 255) / 256;
  if (gr > 65536) gr = 65536;
  hipLaunchKernelGGL(k_state_gamma, dim3(unsigned(gr)), dim3(256), 0, s, sab, sab64 ? 1 : 0, sum_a,
                     sum_b, n, pa, pb, layout, gamma, gamma_f32, numer);
  return hipGetLastError();
}

}  // namespace cpi
