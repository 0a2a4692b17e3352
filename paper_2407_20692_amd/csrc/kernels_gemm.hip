// Sum of products S_ab = A^T B on matrix cores (int8 or FP4 operands),
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
//
// Bit rows can instead feed the FP4 matrix-core op
// (v_mfma_f32_16x16x128_f8f6f4 with E2M1 operands, no block scales).  Word w
// of a lane supplies the lane's 32 K values of one such op: nibble k of
// dword d holds frame 4k + d of the word.  A single set bit is an exact
// E2M1 value (bit 0: 0.5, bit 1: 1, bit 2: 2), so a dword can often be cut
// out of the word with one AND: the N operand takes dwords 0, 1, 2 as
// w & 0x1..., w & 0x2..., w & 0x4... (values 0.5, 1, 2), and the M rows are
// stored with bits 0 and 2 of every 4-bit group exchanged, so the same ANDs
// give it values 2, 1, 0.5 for the same frames.  Frame 4k + 3 sits on the
// sign bit and is shifted to bit 1 (value 1) on both sides.  Every product
// of two set bits is then exactly 1, the FP32 accumulator holds integers
// exactly up to 2^24, and the sums equal the int8 ones bit for bit as long
// as one launch covers at most 2^24 frames.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "kernels.h"

namespace cpi {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Scale operands 0 select the unscaled form of the op (plain products),
// which issues faster than the block-scaled one.
constexpr int kNoScale = 0;
constexpr int kFmtE2M1 = 4;

// The four E2M1 dwords (32 K values) of bit word x of an N row (plain
// layout: frames 4k + 0, 1, 2 at values 0.5, 1, 2; frame 4k + 3 at 1) ...
__device__ __forceinline__ v8i fp4_operand_n(uint32_t x) {
  return v8i{int(x & 0x11111111u), int(x & 0x22222222u), int(x & 0x44444444u),
             int((x >> 2) & 0x22222222u), 0, 0, 0, 0};
}
// ... and of an M row stored with bits 0 and 2 of each group exchanged
// (frames 4k + 0, 1, 2 at values 2, 1, 0.5; frame 4k + 3 at 1).
__device__ __forceinline__ v8i fp4_operand_m(uint32_t x) {
  return v8i{int(x & 0x44444444u), int(x & 0x22222222u), int(x & 0x11111111u),
             int((x >> 2) & 0x22222222u), 0, 0, 0, 0};
}

// Work-group b executes on XCD b % 8.  Give each XCD a contiguous range of
// output tiles so that tiles sharing operand rows share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
  const int per = nwg >> 3, rem = nwg & 7;
  const int x = b & 7, i = b >> 3;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + i;
}

// Tile of work-group b: XCD-contiguous ranges, walked in groups of 8 tile
// rows, so that the work-groups resident on one XCD at a time cover about
// 8 x 8 tiles and re-use each other's operand rows in its L2.
__device__ __forceinline__ void tile_of(int b, int nwg, int tiles_m, int* tm, int* tn) {
  constexpr int kGroup = 8;
  const int id = xcd_remap(b, nwg);
  const int tiles_n = nwg / tiles_m;
  const int per_group = kGroup * tiles_n;
  const int grp = id / per_group;
  const int m0 = grp * kGroup;
  const int gm = (tiles_m - m0) < kGroup ? (tiles_m - m0) : kGroup;
  const int in = id - grp * per_group;
  *tm = m0 + in % gm;
  *tn = in / gm;
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
  if (g.gamma) __builtin_nontemporal_store(gam, g.gamma + idx);
  if (g.gamma_f32) __builtin_nontemporal_store(float(gam), g.gamma_f32 + idx);
  if (g.numer) __builtin_nontemporal_store(numer, g.numer + idx);
}

// Four consecutive detector-A pixels p..p+3 of view q, s[] in the operand
// domain without offset (bit operands).  Vector loads and stores when the
// quad is whole and 16-byte aligned in view-major order, else per element.
template <int MODE>
__device__ __forceinline__ void store_quad(const Epi& g, int64_t q, int64_t p, const int32_t (&s)[4],
                                           bool vec) {
  if (!vec) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (p + k < g.pa) store_result<MODE>(g, q, p + k, int64_t(s[k]), 0);
    return;
  }
  const int64_t idx_vm = q * g.pa + p;
  int64_t t[4];
  if constexpr (MODE == EPI_STREAM32) {
    int4 a = *reinterpret_cast<const int4*>(g.acc32 + idx_vm);
    a.x += s[0];
    a.y += s[1];
    a.z += s[2];
    a.w += s[3];
    *reinterpret_cast<int4*>(g.acc32 + idx_vm) = a;
    t[0] = a.x;
    t[1] = a.y;
    t[2] = a.z;
    t[3] = a.w;
  } else if constexpr (MODE == EPI_STREAM64) {
    longlong2 a0 = *reinterpret_cast<const longlong2*>(g.acc64 + idx_vm);
    longlong2 a1 = *reinterpret_cast<const longlong2*>(g.acc64 + idx_vm + 2);
    a0.x += s[0];
    a0.y += s[1];
    a1.x += s[2];
    a1.y += s[3];
    *reinterpret_cast<longlong2*>(g.acc64 + idx_vm) = a0;
    *reinterpret_cast<longlong2*>(g.acc64 + idx_vm + 2) = a1;
    t[0] = a0.x;
    t[1] = a0.y;
    t[2] = a1.x;
    t[3] = a1.y;
  } else {
    static_assert(MODE == EPI_FINAL, "quad epilogue modes");
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = s[k];
  }
  const int64_t n = g.n;
  const int64_t sb = g.sum_b[q];
  const longlong2 sa01 = *reinterpret_cast<const longlong2*>(g.sum_a + p);
  const longlong2 sa23 = *reinterpret_cast<const longlong2*>(g.sum_a + p + 2);
  const int64_t sa[4] = {sa01.x, sa01.y, sa23.x, sa23.y};
  const double nn = double(n) * double(n);
  int64_t num[4];
  double gam[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    num[k] = n * t[k] - sa[k] * sb;
    gam[k] = double(num[k]) / nn;
  }
  // The outputs are written once and not read back here: non-temporal
  // stores stream them past the caches, which keep the operand rows (at
  // 65536 x 65536 pairs this cut the contraction from 18.4 to 12.0 ms).
  typedef double d2v __attribute__((ext_vector_type(2)));
  typedef float f4v __attribute__((ext_vector_type(4)));
  typedef int64_t l2v __attribute__((ext_vector_type(2)));
  if (g.layout == CPI_GAMMA_VIEW_MAJOR) {
    if (g.gamma) {
      __builtin_nontemporal_store(d2v{gam[0], gam[1]}, reinterpret_cast<d2v*>(g.gamma + idx_vm));
      __builtin_nontemporal_store(d2v{gam[2], gam[3]},
                                  reinterpret_cast<d2v*>(g.gamma + idx_vm + 2));
    }
    if (g.gamma_f32)
      __builtin_nontemporal_store(f4v{float(gam[0]), float(gam[1]), float(gam[2]), float(gam[3])},
                                  reinterpret_cast<f4v*>(g.gamma_f32 + idx_vm));
    if (g.numer) {
      __builtin_nontemporal_store(l2v{num[0], num[1]}, reinterpret_cast<l2v*>(g.numer + idx_vm));
      __builtin_nontemporal_store(l2v{num[2], num[3]},
                                  reinterpret_cast<l2v*>(g.numer + idx_vm + 2));
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t idx = (p + k) * g.pb + q;
      if (g.gamma) __builtin_nontemporal_store(gam[k], g.gamma + idx);
      if (g.gamma_f32) __builtin_nontemporal_store(float(gam[k]), g.gamma_f32 + idx);
      if (g.numer) __builtin_nontemporal_store(num[k], g.numer + idx);
    }
  }
}

template <int FM, int FN, bool BITS, int MODE, bool F4 = false>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  static_assert(BITS || !F4, "FP4 operands come from bit rows");
  if (g.cond) {
    const uint32_t mx = g.stats[0];
    if ((g.cond == 1) != (mx <= 1u)) return;
  }
  constexpr int WM = 16 * FM, WN = 16 * FN;
  const int tiles_m = int(g.m_pad / (2 * WM));
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, &tm, &tn);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, kg = lane >> 4;
  const int64_t m0 = int64_t(tm) * (2 * WM) + (wave & 1) * WM;
  const int64_t n0 = int64_t(tn) * (2 * WN) + (wave >> 1) * WN;
  const uint8_t* pm = g.opm + (m0 + r) * g.row_bytes + g.k_byte_off + kg * 16;
  const uint8_t* pn = g.opn + (n0 + r) * g.row_bytes + g.k_byte_off + kg * 16;
  const int64_t fstride = 16 * g.row_bytes;

  using Acc = std::conditional_t<F4, v4f, v4i>;
  Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  v4i am[FM], bn[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) am[i] = *reinterpret_cast<const v4i*>(pm + i * fstride);
#pragma unroll
  for (int j = 0; j < FN; ++j) bn[j] = *reinterpret_cast<const v4i*>(pn + j * fstride);

  for (int64_t kb = 0; kb < g.kblocks; ++kb) {
    // next block's operands, loaded while this block is multiplied
    const int64_t nx = (kb + 1 < g.kblocks ? kb + 1 : kb) * 64;
    v4i am2[FM], bn2[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) am2[i] = *reinterpret_cast<const v4i*>(pm + i * fstride + nx);
#pragma unroll
    for (int j = 0; j < FN; ++j) bn2[j] = *reinterpret_cast<const v4i*>(pn + j * fstride + nx);

    if constexpr (F4) {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        v8i ea[FM], eb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) ea[i] = fp4_operand_m(uint32_t(am[i][w]));
#pragma unroll
        for (int j = 0; j < FN; ++j) eb[j] = fp4_operand_n(uint32_t(bn[j][w]));
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                ea[i], eb[j], acc[i][j], kFmtE2M1, kFmtE2M1, 0, kNoScale, 0, kNoScale);
      }
    } else if constexpr (BITS) {
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
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(am[i], bn[j], acc[i][j], 0, 0, 0);
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

// ---- Bit-row contraction fed through an LDS pipeline ----------------------
// FP4 (k_gemm_f4lds) or int8 (k_gemm_i8lds) matrix-core ops on bit rows, with
// the expansions of the register-fed kernel above.
// A work-group computes a 128 x 128 tile (2 x 2 waves of 64 x 64).  Each
// 512-frame block needs 256 operand rows x 64 bytes = 16 KB, which direct
// global->LDS copies (no registers) bring into one of S stages, S - 1 blocks
// ahead of the block being multiplied; one barrier per block.  Each row
// segment is fetched once per work-group.
//
// Stage layout: 16 groups of 16 rows (groups 0-7: M rows, 8-15: N rows),
// 1 KB each, one copy instruction per group.  Chunk c (16 bytes) of row r of
// a group sits at slot 4r + (c ^ ((r >> 2) & 3)), so the 16 lanes reading one
// chunk column of a fragment touch 16 distinct 4-bank groups.
//
// LDS reads are issued by inline asm: the compiler would otherwise wait for
// every outstanding global->LDS copy before each LDS read, serializing the
// pipeline.  Ordering is explicit instead: each wave waits for its own copies
// of the block (vmcnt), then a barrier makes every wave's copies visible and
// guarantees that the stage about to be refilled has been read by all waves.
typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Eight 16-byte LDS reads and the wait for them, as one unit.
__device__ __forceinline__ void lds_read8(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3,
                                          uint32_t a4, uint32_t a5, uint32_t a6, uint32_t a7,
                                          v4i (&x)[4], v4i (&y)[4]) {
  asm volatile(
      "ds_read_b128 %0, %8\n"
      "ds_read_b128 %1, %9\n"
      "ds_read_b128 %2, %10\n"
      "ds_read_b128 %3, %11\n"
      "ds_read_b128 %4, %12\n"
      "ds_read_b128 %5, %13\n"
      "ds_read_b128 %6, %14\n"
      "ds_read_b128 %7, %15\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(y[0]), "=&v"(y[1]),
        "=&v"(y[2]), "=&v"(y[3])
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4), "v"(a5), "v"(a6), "v"(a7));
}

template <int S>
__device__ __forceinline__ void wait_copies() {
  // s_waitcnt vmcnt(4 * (S - 2)), expcnt and lgkmcnt left open
  static_assert(S >= 2 && 4 * (S - 2) < 16, "stage count");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (4 * (S - 2)));
}

// __launch_bounds__(256, 2) makes the compiler fit the kernel in about 168
// registers (no spills), so that three work-groups share a CU (the LDS limit):
// measured 12% faster than its unconstrained allocation (240 registers, two
// work-groups) on Da 128 x 128, Db 64 x 64, 20000 frames.
constexpr int kLdsStage = 16384;   // bytes per stage

template <int MODE, int S, bool I8>
__device__ __forceinline__ void gemm_lds(const GemmArgs& g, uint8_t* stage) {
  if (g.cond) {
    const uint32_t mx = g.stats[0];
    if ((g.cond == 1) != (mx <= 1u)) return;
  }
  constexpr int kStage = kLdsStage;
  const int tiles_m = int(g.m_pad / 128);
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, &tm, &tn);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t mb = int64_t(tm) * 128, nb = int64_t(tn) * 128;

  // copy side: waves 0-1 copy the 128 M rows, waves 2-3 the 128 N rows, 64
  // rows (4 groups) each; lane -> (row, chunk) within a group
  const int cr = lane >> 2;
  const int cc = (lane & 3) ^ ((cr >> 2) & 3);
  const uint8_t* wbase = wave < 2 ? g.opm + (mb + 64 * wave) * g.row_bytes
                                  : g.opn + (nb + 64 * (wave - 2)) * g.row_bytes;
  // wave-uniform base + 32-bit lane offset (scalar-base addressing)
  const uint8_t* ubase = wbase + g.k_byte_off;
  const uint32_t loff = uint32_t(cr * g.row_bytes + 16 * cc);
  const int64_t gstride = 16 * g.row_bytes;
  const uint32_t lds0 = uint32_t(reinterpret_cast<uintptr_t>(stage));
  auto copy_block = [&](int64_t kb, int st) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      __builtin_amdgcn_global_load_lds(ubase + (q * gstride + kb * 64) + loff,
                                       (lds_ptr_t)(stage + st * kStage + (wave * 4 + q) * 1024),
                                       16, 0, 0);
  };

  // read side
  const int wm = wave & 1, wn = wave >> 1;
  const int r = lane & 15, kg = lane >> 4;
  const uint32_t roff = uint32_t(r * 64 + 16 * (kg ^ ((r >> 2) & 3)));

  using Acc = std::conditional_t<I8, v4i, v4f>;
  Acc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  const int64_t last = g.kblocks - 1;
#pragma unroll
  for (int p = 0; p < S - 1; ++p) copy_block(p < last ? p : last, p);

  int st = 0;
  for (int64_t kb = 0; kb < g.kblocks; ++kb) {
    wait_copies<S>();
    __builtin_amdgcn_s_barrier();
    {
      const int64_t nxt = kb + S - 1;
      const int ns = st == 0 ? S - 1 : st - 1;   // (kb + S - 1) % S
      copy_block(nxt < last ? nxt : last, ns);
    }
    const uint32_t base = lds0 + uint32_t(st * kStage) + roff;
    const uint32_t ba = base + wm * 4096, bb = base + 8192 + wn * 4096;
    v4i am[4], bn[4];
    lds_read8(ba, ba + 1024, ba + 2048, ba + 3072, bb, bb + 1024, bb + 2048, bb + 3072, am, bn);
    if constexpr (I8) {
      const int mask = 0x01010101;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          v4i ea[4], eb[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t x = uint32_t(am[i][w]);
            ea[i] = v4i{int((x >> (4 * h + 0)) & mask), int((x >> (4 * h + 1)) & mask),
                        int((x >> (4 * h + 2)) & mask), int((x >> (4 * h + 3)) & mask)};
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t x = uint32_t(bn[j][w]);
            eb[j] = v4i{int((x >> (4 * h + 0)) & mask), int((x >> (4 * h + 1)) & mask),
                        int((x >> (4 * h + 2)) & mask), int((x >> (4 * h + 3)) & mask)};
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ea[i], eb[j], acc[i][j], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        v8i ea[4], eb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ea[i] = fp4_operand_m(uint32_t(am[i][w]));
#pragma unroll
        for (int j = 0; j < 4; ++j) eb[j] = fp4_operand_n(uint32_t(bn[j][w]));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                ea[i], eb[j], acc[i][j], kFmtE2M1, kFmtE2M1, 0, kNoScale, 0, kNoScale);
      }
    }
    st = st == S - 1 ? 0 : st + 1;
  }
  // the last copies (clamped repeats of the final block) are still in flight;
  // every wave must also be done with the stages before they are reused
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();

  // Epilogue through LDS, one half of the tile (64 rows) at a time: the two
  // waves owning those rows store their sums (exact integers) into a padded
  // row-major tile, then every thread finishes four consecutive columns of
  // one row, so that state and output accesses are contiguous vectors.
  constexpr int kPitch = 132;   // ints per staged row: 128 + 4 (bank spread)
  static_assert(64 * kPitch * 4 <= S * kStage, "epilogue tile fits the stages");
  int32_t* tile = reinterpret_cast<int32_t*>(stage);
  const Epi e{g.mode,   g.layout, g.pa,        g.pb,    g.n,     g.kchunk, g.sum_a, g.sum_b,
              g.csum_a, g.csum_b, g.gamma,     g.gamma_f32, g.numer, g.acc64,  g.acc32};
  const bool vec = (g.pa & 3) == 0;
  const int t = threadIdx.x;
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    if (wm == h) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            tile[(16 * i + 4 * kg + u) * kPitch + wn * 64 + 16 * j + r] = int32_t(acc[i][j][u]);
    }
    __syncthreads();
#pragma unroll 1
    for (int step = 0; step < 8; ++step) {
      const int row = step * 8 + (t >> 5);
      const int cq = (t & 31) * 4;
      const int64_t q = mb + 64 * h + row;
      const int64_t p = nb + cq;
      const int4 v = *reinterpret_cast<const int4*>(tile + row * kPitch + cq);
      const int32_t sv[4] = {v.x, v.y, v.z, v.w};
      if (q < e.pb && p < e.pa) store_quad<MODE>(e, q, p, sv, vec);
    }
    __syncthreads();
  }
}

template <int MODE, int S>
__global__ __launch_bounds__(256, 2) void k_gemm_f4lds(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint8_t stage[S * kLdsStage];
  gemm_lds<MODE, S, false>(g, stage);
}

template <int MODE, int S>
__global__ __launch_bounds__(256, 2) void k_gemm_i8lds(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint8_t stage[S * kLdsStage];
  gemm_lds<MODE, S, true>(g, stage);
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
    if (gamma) __builtin_nontemporal_store(gam, gamma + idx);
    if (gamma_f32) __builtin_nontemporal_store(float(gam), gamma_f32 + idx);
    if (numer) __builtin_nontemporal_store(num, numer + idx);
  }
}

// CPI_GEMM_FEED=regs selects the register-fed kernels for bit rows
// (measurement runs); the default feeds the matrix cores through the LDS
// pipeline.
bool fp4_from_registers() {
  static const bool on = [] {
    const char* v = std::getenv("CPI_GEMM_FEED");
    return v && std::strcmp(v, "regs") == 0;
  }();
  return on;
}

template <int FM, int FN, bool BITS, int MODE, bool F4 = false>
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles_m = a.m_pad / (32 * FM);
  const int64_t tiles_n = a.n_pad / (32 * FN);
  if (tiles_m * (32 * FM) != a.m_pad || tiles_n * (32 * FN) != a.n_pad) return hipErrorInvalidValue;
  const int64_t nwg = tiles_m * tiles_n;
  if (nwg <= 0 || nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<FM, FN, BITS, MODE, F4>), dim3(unsigned(nwg)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Matrix-core encoding of bit rows (CPI_MMA_AUTO or CPI_MMA_INT8), process-wide.
std::atomic<int> g_mma_encoding{[] {
  const char* v = std::getenv("CPI_GEMM_ENC");
  return (v && std::strcmp(v, "int8") == 0) ? int(CPI_MMA_INT8) : int(CPI_MMA_AUTO);
}()};

bool fp4_enabled() { return g_mma_encoding.load(std::memory_order_relaxed) == CPI_MMA_AUTO; }

constexpr int64_t kFp4MaxFrames = int64_t(1) << 24;

template <int MODE, int S, bool I8>
hipError_t launch_lds(const GemmArgs& a, hipStream_t s) {
  const int64_t tiles_m = a.m_pad / 128, tiles_n = a.n_pad / 128;
  if (tiles_m * 128 != a.m_pad || tiles_n * 128 != a.n_pad || a.kblocks < 1)
    return hipErrorInvalidValue;
  const int64_t nwg = tiles_m * tiles_n;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  if constexpr (I8)
    hipLaunchKernelGGL((k_gemm_i8lds<MODE, S>), dim3(unsigned(nwg)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_gemm_f4lds<MODE, S>), dim3(unsigned(nwg)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_bits(const GemmArgs& a, hipStream_t s) {
  if (a.fp4) {
    if (a.kblocks * 512 > kFp4MaxFrames) return hipErrorInvalidValue;
    if (fp4_from_registers()) return launch_gemm<4, 4, true, MODE, true>(a, s);
    return launch_lds<MODE, 3, false>(a, s);
  }
  if (fp4_from_registers()) return launch_gemm<4, 4, true, MODE>(a, s);
  return launch_lds<MODE, 3, true>(a, s);
}

}  // namespace

hipError_t gemm_correlate(const GemmArgs& a, bool bits, hipStream_t s) {
  switch (a.mode) {
    case EPI_FINAL:
      return bits ? launch_bits<EPI_FINAL>(a, s) : launch_gemm<4, 4, false, EPI_FINAL>(a, s);
    case EPI_STREAM32:
      return bits ? launch_bits<EPI_STREAM32>(a, s)
                  : launch_gemm<4, 4, false, EPI_STREAM32>(a, s);
    case EPI_FINAL_ACC64:
      return launch_gemm<4, 4, false, EPI_FINAL_ACC64>(a, s);
    case EPI_STORE64:
      return launch_gemm<4, 4, false, EPI_STORE64>(a, s);
    case EPI_ADD64:
      return launch_gemm<4, 4, false, EPI_ADD64>(a, s);
    case EPI_STREAM64:
      return bits ? launch_bits<EPI_STREAM64>(a, s)
                  : launch_gemm<4, 4, false, EPI_STREAM64>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

bool bits_use_fp4(int64_t kblocks) { return fp4_enabled() && kblocks * 512 <= kFp4MaxFrames; }

void set_mma_encoding(int enc) { g_mma_encoding.store(enc, std::memory_order_relaxed); }
int get_mma_encoding() { return g_mma_encoding.load(std::memory_order_relaxed); }

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
