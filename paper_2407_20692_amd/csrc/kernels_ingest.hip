// Ingest: frame-major detector frames -> pixel-major contraction operands.
//
// The sums of Eq. (1) run over frames, so the contraction dimension of
// S_ab = A^T B is the frame index.  Matrix-core operands want that dimension
// contiguous per pixel, so every frame block is transposed once here:
//   * binary frames become bit rows: bit j of 32-bit word w of row p is the
//     value of pixel p in frame 32*w + j (the paper's bit packing, Section 4.1);
//   * other byte frames become int8 rows, offset by -128 when a value exceeds
//     127 (this leaves the numerator of Eq. (1) unchanged).
// Per-pixel sums S_a, S_b are produced on the way.  Frames beyond n and
// pixels beyond npix read as zero, so padded rows and columns contribute
// nothing to any product.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "kernels.h"

namespace cpi {

namespace {

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t count, uint32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t count, uint64_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Zeroes up to kZeroRanges ranges of 64-bit words in one launch; block row
// blockIdx.y takes range blockIdx.y.
__global__ void k_zero_ranges(ZeroRanges z) {
  const int k = blockIdx.y;
  if (k >= z.count) return;
  uint64_t* __restrict__ p = z.ptr[k];
  const int64_t n = z.words[k];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

__global__ void k_add_i64(int64_t* __restrict__ dst, const int64_t* __restrict__ src,
                          int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] += src[i];
}

// Lane-indexed insert of a wave-uniform value: lane L of `old` becomes v
// (v_writelane_b32 through its LLVM intrinsic, so that the compiler knows the
// operation).  Callers keep it out of divergent control flow: every lane of
// the wave is active wherever it is used.
extern "C" __device__ uint32_t cpi_llvm_writelane(uint32_t v, uint32_t lane, uint32_t old) __asm(
    "llvm.amdgcn.writelane.i32");

template <int L>
__device__ __forceinline__ uint32_t write_lane(uint32_t old, uint32_t v) {
  return cpi_llvm_writelane(v, uint32_t(L), old);
}

// Bit of pixel J (0..127) in this lane's 16 packed bytes of one frame.
template <int J>
__device__ __forceinline__ uint32_t pixel_bit(const uint32_t (&d)[4]) {
  return (d[J >> 5] >> (J & 31)) & 1u;
}

// One ballot per pixel J: bit l of the result is pixel J in frame f0 + l.
// Pixel J's 64 frame bits go to lane J % 64, words 2*SUB, 2*SUB+1 of half J/64.
template <int SUB, int J, int ND>
__device__ __forceinline__ void ballot_pixel(const uint32_t (&d)[ND], uint32_t (&w0)[16],
                                             uint32_t (&w1)[16]) {
  const unsigned long long m = __ballot(pixel_bit<J>(d));
  const uint32_t lo = uint32_t(m), hi = uint32_t(m >> 32);
  if constexpr (J < 64) {
    w0[2 * SUB] = write_lane<J>(w0[2 * SUB], lo);
    w0[2 * SUB + 1] = write_lane<J>(w0[2 * SUB + 1], hi);
  } else {
    w1[2 * SUB] = write_lane<J - 64>(w1[2 * SUB], lo);
    w1[2 * SUB + 1] = write_lane<J - 64>(w1[2 * SUB + 1], hi);
  }
}

template <int SUB, int ND, int... J>
__device__ __forceinline__ void ballot_all(const uint32_t (&d)[ND], uint32_t (&w0)[16],
                                           uint32_t (&w1)[16], std::integer_sequence<int, J...>) {
  (ballot_pixel<SUB, J, ND>(d, w0, w1), ...);
}

// Loads the lane's frame data for sub-block SUB and transposes it.
template <int SUB, int ND, typename Load>
__device__ __forceinline__ void transpose_sub(Load&& load, uint32_t (&w0)[16],
                                              uint32_t (&w1)[16]) {
  uint32_t d[ND];
  load(SUB, d);
  ballot_all<SUB, ND>(d, w0, w1, std::make_integer_sequence<int, 128>{});
}

template <int ND, typename Load, int... S>
__device__ __forceinline__ void transpose_block(Load&& load, uint32_t (&w0)[16],
                                                uint32_t (&w1)[16],
                                                std::integer_sequence<int, S...>) {
  (transpose_sub<S, ND>(load, w0, w1), ...);
}

// Exchange bits 0 and 2 of every 4-bit group.
__device__ __forceinline__ uint32_t swap_bits02(uint32_t x) {
  return (x & 0xAAAAAAAAu) | ((x & 0x11111111u) << 2) | ((x >> 2) & 0x11111111u);
}

unsigned grid_for(int64_t count, int threads) {
  int64_t g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return unsigned(g);
}

// Packed-bit frames -> bit rows.  One wave owns 128 pixels and a slice of
// 512-frame blocks.  Lane l reads the 16 bytes (128 pixels) of frame
// f0 + l; one wave ballot per pixel then yields that pixel's 64 frame bits,
// which a lane select drops into the register of the lane that owns the pixel
// (pixel j -> lane j % 64, half j / 64).
__global__ __launch_bounds__(64) void k_ingest_bits(IngestJob j0, IngestJob j1, int64_t groups0,
                                                   int64_t n, int64_t kw, int64_t nblocks,
                                                   int64_t blocks_per_slice) {
  // work-groups [0, groups0) take detector job j0, the rest job j1
  const bool second = int64_t(blockIdx.x) >= groups0;
  const uint8_t* __restrict__ frames = second ? j1.frames : j0.frames;
  const int64_t fbytes = ((second ? j1.npix : j0.npix) + 7) / 8;
  uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(second ? j1.out : j0.out);
  unsigned long long* __restrict__ sums =
      reinterpret_cast<unsigned long long*>(second ? j1.sums : j0.sums);
  const int swap02 = second ? j1.swap02 : j0.swap02;
  const int lane = threadIdx.x;
  const int64_t p0 = (int64_t(blockIdx.x) - (second ? groups0 : 0)) * 128;
  const int64_t byte0 = p0 >> 3;
  const int64_t kb0 = int64_t(blockIdx.y) * blocks_per_slice;
  int64_t kb1 = kb0 + blocks_per_slice;
  if (kb1 > nblocks) kb1 = nblocks;
  const bool vec = ((fbytes & 15) == 0) && (byte0 + 16 <= fbytes);
  unsigned long long s0 = 0, s1 = 0;
  for (int64_t kb = kb0; kb < kb1; ++kb) {
    uint32_t w0[16], w1[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      w0[i] = 0;
      w1[i] = 0;
    }
    // Branch-free: frames beyond n and bytes beyond the frame read valid
    // addresses and are masked to zero, so the wave stays fully active.
    auto load = [&](int sub, uint32_t(&d)[4]) {
      const int64_t f = kb * 512 + sub * 64 + lane;
      const bool fin = f < n;
      const uint8_t* src = frames + (fin ? f : 0) * fbytes;
      const uint32_t m = fin ? 0xffffffffu : 0u;
      if (vec) {
        const uint4 v = *reinterpret_cast<const uint4*>(src + byte0);
        d[0] = v.x & m;
        d[1] = v.y & m;
        d[2] = v.z & m;
        d[3] = v.w & m;
      } else {
        d[0] = d[1] = d[2] = d[3] = 0u;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          const bool ok = byte0 + b < fbytes;
          const uint32_t x = src[ok ? byte0 + b : 0];
          d[b >> 2] |= (ok ? x : 0u) << (8 * (b & 3));
        }
        d[0] &= m;
        d[1] &= m;
        d[2] &= m;
        d[3] &= m;
      }
    };
    transpose_block<4>(load, w0, w1, std::make_integer_sequence<int, 8>{});
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      s0 += __popc(w0[i]);
      s1 += __popc(w1[i]);
      if (swap02) {
        w0[i] = swap_bits02(w0[i]);
        w1[i] = swap_bits02(w1[i]);
      }
    }
    uint4* o0 = reinterpret_cast<uint4*>(out + (p0 + lane) * kw + kb * 16);
    uint4* o1 = reinterpret_cast<uint4*>(out + (p0 + 64 + lane) * kw + kb * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      o0[q] = make_uint4(w0[4 * q], w0[4 * q + 1], w0[4 * q + 2], w0[4 * q + 3]);
      o1[q] = make_uint4(w1[4 * q], w1[4 * q + 1], w1[4 * q + 2], w1[4 * q + 3]);
    }
  }
  atomicAdd(&sums[p0 + lane], s0);
  atomicAdd(&sums[p0 + 64 + lane], s1);
}

// Byte frames -> bit rows.  Each wave owns 256 consecutive pixels (lane l:
// pixels 4l .. 4l+3, one dword of every frame row, so a wave reads 256
// contiguous bytes per frame) and a slice of 128-frame units.  The low bits
// of 8 frames are gathered into one byte per pixel (frame j of the 8 at bit
// j: a mask and a shift-or per frame); four such octets are then regrouped
// byte-wise into the 32-bit row words of the 4 pixels.  The OR of all bytes
// goes to stats[0], so the rows (and the popcount sums) are valid exactly
// when that OR is at most 1.
__device__ __forceinline__ void bytes_transpose4(const uint32_t (&t)[4], uint32_t (&w)[4]) {
  // w[k] byte o = t[o] byte k
#pragma unroll
  for (int k = 0; k < 4; ++k)
    w[k] = ((t[0] >> (8 * k)) & 0xffu) | (((t[1] >> (8 * k)) & 0xffu) << 8) |
           (((t[2] >> (8 * k)) & 0xffu) << 16) | (((t[3] >> (8 * k)) & 0xffu) << 24);
}

template <bool ALIGNED>
__global__ __launch_bounds__(256) void k_u8_to_bits(IngestJob j0, IngestJob j1, int64_t groups0,
                                                    int64_t n, int64_t kw, int64_t nunits,
                                                    int64_t units_per_slice,
                                                    uint32_t* __restrict__ stats) {
  // work-groups [0, groups0) take detector job j0, the rest job j1
  const bool second = int64_t(blockIdx.x) >= groups0;
  const uint8_t* __restrict__ frames = second ? j1.frames : j0.frames;
  const int64_t npix = second ? j1.npix : j0.npix;
  const int64_t npix_pad = second ? j1.npix_pad : j0.npix_pad;
  uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(second ? j1.out : j0.out);
  unsigned long long* __restrict__ sums =
      reinterpret_cast<unsigned long long*>(second ? j1.sums : j0.sums);
  const int swap02 = second ? j1.swap02 : j0.swap02;
  const int64_t blk = int64_t(blockIdx.x) - (second ? groups0 : 0);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t p0 = (blk * 4 + wave) * 256;
  if (p0 >= npix_pad || n <= 0) return;
  const int64_t px = p0 + 4 * lane;
  const int64_t u0 = int64_t(blockIdx.y) * units_per_slice;
  int64_t u1 = u0 + units_per_slice;
  if (u1 > nunits) u1 = nunits;
  uint32_t any = 0;
  uint32_t s[4] = {0u, 0u, 0u, 0u};
  // Lanes whose pixels lie beyond npix read pixel 0 and mask their results
  // (rows, sums, OR) to zero; frames beyond n, in the last block only, read
  // frame 0 and are masked to zero per frame.
  const bool pin = px < npix;
  const uint32_t lane_off = uint32_t(pin ? px : 0);
  const uint32_t pmask = pin ? 0xffffffffu : 0u;
  auto load = [&](int64_t f) -> uint32_t {
    const uint8_t* row = frames + f * npix;
    if constexpr (ALIGNED) {
      return *reinterpret_cast<const uint32_t*>(row + lane_off);
    } else {
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t o = px + b < npix ? uint32_t(px + b) : 0u;
        v |= uint32_t(row[o]) << (8 * b);
      }
      return v;
    }
  };
  // One unit = 128 frames: four 32-bit row words (one 16-byte store) for
  // each of the lane's four pixels.
  auto unit = [&](int64_t u, auto tail) {
    constexpr bool TAIL = decltype(tail)::value;
    {
      uint32_t w[4][4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t f0 = u * 128 + g * 32;
        uint32_t d[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) {
          if constexpr (TAIL) {
            const bool fin = f0 + j < n;
            d[j] = load(fin ? f0 + j : 0) & (fin ? 0xffffffffu : 0u);
          } else {
            d[j] = load(f0 + j);
          }
        }
        uint32_t t[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          uint32_t acc = 0;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            any |= d[8 * o + j];
            acc |= (d[8 * o + j] & 0x01010101u) << j;
          }
          t[o] = acc;
        }
        uint32_t wk[4];
        bytes_transpose4(t, wk);
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k][g] = wk[k] & pmask;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          s[k] += __popc(w[k][g]);
          if (swap02) w[k][g] = swap_bits02(w[k][g]);
        }
        *reinterpret_cast<uint4*>(out + (px + k) * kw + u * 4) =
            make_uint4(w[k][0], w[k][1], w[k][2], w[k][3]);
      }
    }
  };
  for (int64_t u = u0; u < u1; ++u) {
    if (u * 128 + 128 <= n)
      unit(u, std::false_type{});
    else
      unit(u, std::true_type{});
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (s[k]) atomicAdd(&sums[px + k], (unsigned long long)s[k]);
  any &= pmask;
  any = (any | (any >> 8) | (any >> 16) | (any >> 24)) & 0xffu;
  for (int off = 32; off > 0; off >>= 1) any |= __shfl_xor(any, off, 64);
  // Bits of stats[0] only get set during the launch, so a wave whose bits are
  // all present already (read at device scope, not from a stale cache) has
  // nothing to add: this keeps most waves off the single contended word.
  if (lane == 0 && any) {
    const uint32_t cur = __hip_atomic_load(stats, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((cur | any) != cur) atomicOr(stats, any);
  }
}

// Per-pixel byte sums (non-binary data only).  A work-group owns 256
// consecutive pixels: 16 threads cover them 16 bytes each, and the 16 thread
// rows walk interleaved frames of the group's frame slice.  Partial sums are
// reduced in LDS, so each pixel receives one atomic per work-group.
__global__ __launch_bounds__(256) void k_u8_sums(IngestJob j0, IngestJob j1, int64_t groups0, int64_t n,
                                                 int64_t frames_per_slice,
                                                 const uint32_t* __restrict__ stats) {
  if (stats[0] <= 1u) return;
  // work-groups [0, groups0) take detector job j0, the rest job j1
  const bool second = int64_t(blockIdx.x) >= groups0;
  const uint8_t* __restrict__ frames = second ? j1.frames : j0.frames;
  const int64_t npix = second ? j1.npix : j0.npix;
  unsigned long long* __restrict__ sums =
      reinterpret_cast<unsigned long long*>(second ? j1.sums2 : j0.sums2);
  const int64_t blk = int64_t(blockIdx.x) - (second ? groups0 : 0);
  __shared__ uint32_t red[16][256 + 1];
  const int t = threadIdx.x;
  const int col = t & 15, row = t >> 4;
  const int64_t px = blk * 256 + col * 16;
  const int64_t f0 = int64_t(blockIdx.y) * frames_per_slice;
  int64_t f1 = f0 + frames_per_slice;
  if (f1 > n) f1 = n;
  uint32_t s[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) s[b] = 0;
  if (px < npix) {
    const bool vec = ((npix & 15) == 0);
    for (int64_t f = f0 + row; f < f1; f += 16) {
      const uint8_t* src = frames + f * npix + px;
      uint32_t d[4] = {0u, 0u, 0u, 0u};
      if (vec) {
        const uint4 v = *reinterpret_cast<const uint4*>(src);
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
      } else {
        for (int b = 0; b < 16; ++b)
          if (px + b < npix) d[b >> 2] |= uint32_t(src[b]) << (8 * (b & 3));
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) s[b] += (d[b >> 2] >> (8 * (b & 3))) & 0xffu;
    }
  }
#pragma unroll
  for (int b = 0; b < 16; ++b) red[row][col * 16 + b] = s[b];
  __syncthreads();
  const int64_t p = blk * 256 + t;
  unsigned long long tot = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) tot += red[r][t];
  if (p < npix && tot) atomicAdd(&sums[p], tot);
}

__global__ void k_select_i64(int64_t* __restrict__ dst, const int64_t* __restrict__ a,
                             const int64_t* __restrict__ b, int64_t count,
                             const uint32_t* __restrict__ stats, int add) {
  const int64_t* src = stats[0] <= 1u ? a : b;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = add ? dst[i] + src[i] : src[i];
}

// Byte frames -> int8 rows through a 64 x 64 LDS tile (only when some byte
// exceeds 1).  Pads (frames >= n, pixels >= npix) are written as 0, the
// value of "no photon" in the offset domain.  Work-groups stride over the
// tiles, so that for binary data (nothing to do) only a few thousand
// work-groups start and exit.
__global__ __launch_bounds__(256) void k_u8_to_bytes(IngestJob j0, IngestJob j1, int64_t n, int64_t kpad,
                                                     int64_t tiles_p0, int64_t tiles0,
                                                     int64_t tiles_p1, int64_t tiles,
                                                     const uint32_t* __restrict__ stats) {
  const uint32_t mx = stats[0];
  if (mx <= 1u) return;
  const uint32_t xo = mx > 127u ? 0x80u : 0u;
  __shared__ uint8_t tile[64][64 + 4];
  const int t = threadIdx.x;
  // tiles [0, tiles0) belong to detector job j0, the rest to job j1
  for (int64_t tt0 = blockIdx.x; tt0 < tiles; tt0 += gridDim.x) {
    const bool second = tt0 >= tiles0;
    const uint8_t* __restrict__ frames = second ? j1.frames : j0.frames;
    const int64_t npix = second ? j1.npix : j0.npix;
    uint8_t* __restrict__ out = second ? j1.out : j0.out;
    const int64_t tiles_p = second ? tiles_p1 : tiles_p0;
    const int64_t tt = tt0 - (second ? tiles0 : 0);
    const int64_t p0 = (tt % tiles_p) * 64;
    const int64_t f0 = (tt / tiles_p) * 64;
    {
      const int fl = t >> 2, pc = (t & 3) * 16;
      const int64_t f = f0 + fl;
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int64_t p = p0 + pc + b;
        uint32_t v = 0;
        if (f < n && p < npix) v = uint32_t(frames[f * npix + p]) ^ xo;
        tile[fl][pc + b] = uint8_t(v);
      }
    }
    __syncthreads();
    {
      const int pl = t >> 2, fc = (t & 3) * 16;
      uint32_t d[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int b = 0; b < 16; ++b) d[b >> 2] |= uint32_t(tile[fc + b][pl]) << (8 * (b & 3));
      *reinterpret_cast<uint4*>(out + (p0 + pl) * kpad + f0 + fc) =
          make_uint4(d[0], d[1], d[2], d[3]);
    }
    __syncthreads();
  }
}

// Side-by-side sensor frames -> the two detectors' bit frames.  A raw frame
// is frame_h rows of frame_w 1-bit pixels, row-major, pixel (y, x) at bit
// (y*frame_w + x) % 8 of byte (y*frame_w + x) / 8; detector A is the left
// half (columns [0, frame_w/2)), detector B the right half.  The same region
// of interest (roi_w x roi_h at roi_x, roi_y inside each half) is repacked
// for both, 8 output pixels per thread, in the frame format of the rest of
// the library (pixel p of a frame at bit p % 8 of byte p / 8).
__global__ __launch_bounds__(256) void k_split_sbs(const uint8_t* __restrict__ in, int64_t n,
                                                   int64_t in_fbytes, int frame_w, int roi_x,
                                                   int roi_y, int roi_w, int roi_h,
                                                   uint8_t* __restrict__ out_a,
                                                   uint8_t* __restrict__ out_b,
                                                   int64_t out_fbytes) {
  const int64_t per_side = n * out_fbytes;
  const int64_t npix = int64_t(roi_w) * roi_h;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < 2 * per_side;
       i += int64_t(gridDim.x) * 256) {
    const bool right = i >= per_side;
    const int64_t local = right ? i - per_side : i;
    const int64_t f = local / out_fbytes, ob = local - f * out_fbytes;
    const uint8_t* src = in + f * in_fbytes;
    const int64_t x_off = (right ? frame_w / 2 : 0) + roi_x;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t p = ob * 8 + k;
      if (p < npix) {
        const int64_t y = p / roi_w, x = p - y * roi_w;
        const int64_t bit = (roi_y + y) * frame_w + x_off + x;
        v |= uint32_t((src[bit >> 3] >> (bit & 7)) & 1u) << k;
      }
    }
    (right ? out_b : out_a)[f * out_fbytes + ob] = uint8_t(v);
  }
}

int64_t slices_for(int64_t groups, int64_t nblocks, int64_t target_waves) {
  int64_t s = (target_waves + groups - 1) / groups;
  if (s < 1) s = 1;
  if (s > nblocks) s = nblocks;
  if (s > 65535) s = 65535;
  return s;
}

}  // namespace

hipError_t fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t fill_u64(uint64_t* p, int64_t count, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t zero_ranges(const ZeroRanges& z, hipStream_t s) {
  if (z.count < 1 || z.count > kZeroRanges) return hipErrorInvalidValue;
  int64_t most = 0;
  for (int k = 0; k < z.count; ++k) most = z.words[k] > most ? z.words[k] : most;
  if (most < 1) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ranges, dim3(grid_for(most, 256), unsigned(z.count)), dim3(256), 0, s,
                     z);
  return hipGetLastError();
}

hipError_t add_i64(int64_t* dst, const int64_t* src, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_add_i64, dim3(grid_for(count, 256)), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}

hipError_t ingest_bits(const IngestJob& a, const IngestJob& b, int64_t n, int64_t kpad_bits,
                       hipStream_t s) {
  // a work-group covers 128 rows: the padded row counts must be multiples of it
  for (const IngestJob* j : {&a, &b})
    if (j->npix_pad % 128 != 0 || j->npix_pad < j->npix) return hipErrorInvalidValue;
  const int64_t groups0 = a.npix_pad / 128;
  const int64_t groups = groups0 + b.npix_pad / 128;
  const int64_t nblocks = kpad_bits / 512;
  const int64_t slices = slices_for(groups, nblocks, 8192);
  const int64_t bps = (nblocks + slices - 1) / slices;
  const int64_t used = (nblocks + bps - 1) / bps;
  if (groups > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ingest_bits, dim3(unsigned(groups), unsigned(used)), dim3(64), 0, s, a, b,
                     groups0, n, kpad_bits / 32, nblocks, bps);
  return hipGetLastError();
}

hipError_t u8_sums(const IngestJob& a, const IngestJob& b, int64_t n, const uint32_t* stats,
                   hipStream_t s) {
  const int64_t groups0 = (a.npix + 255) / 256;
  const int64_t groups = groups0 + (b.npix + 255) / 256;
  int64_t slices = (2048 + groups - 1) / groups;
  if (slices > (n + 15) / 16) slices = (n + 15) / 16;
  if (slices < 1) slices = 1;
  int64_t fps = (n + slices - 1) / slices;
  // a thread row adds at most fps/16 bytes of <= 255 per pixel in uint32
  if (fps > (int64_t(1) << 27)) fps = int64_t(1) << 27;
  slices = (n + fps - 1) / fps;
  if (slices > 65535 || groups > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_u8_sums, dim3(unsigned(groups), unsigned(slices)), dim3(256), 0, s, a, b,
                     groups0, n, fps, stats);
  return hipGetLastError();
}

hipError_t select_i64(int64_t* dst, const int64_t* from_bits, const int64_t* from_bytes,
                      int64_t count, const uint32_t* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_select_i64, dim3(grid_for(count, 256)), dim3(256), 0, s, dst, from_bits,
                     from_bytes, count, stats, 0);
  return hipGetLastError();
}

hipError_t add_select_i64(int64_t* dst, const int64_t* from_bits, const int64_t* from_bytes,
                          int64_t count, const uint32_t* stats, hipStream_t s) {
  hipLaunchKernelGGL(k_select_i64, dim3(grid_for(count, 256)), dim3(256), 0, s, dst, from_bits,
                     from_bytes, count, stats, 1);
  return hipGetLastError();
}

hipError_t u8_to_bits(const IngestJob& a, const IngestJob& b, int64_t n, int64_t kpad_bits,
                      uint32_t* stats, hipStream_t s) {
  // a wave covers 256 rows: the padded row counts must be multiples of it
  for (const IngestJob* j : {&a, &b})
    if (j->npix_pad % 256 != 0 || j->npix_pad < j->npix) return hipErrorInvalidValue;
  const int64_t groups0 = (a.npix_pad / 256 + 3) / 4;
  const int64_t groups = groups0 + (b.npix_pad / 256 + 3) / 4;
  const int64_t waves = (a.npix_pad + b.npix_pad) / 256;
  const int64_t nunits = kpad_bits / 128;
  const int64_t slices = slices_for(waves, nunits, 8192);
  const int64_t ups = (nunits + slices - 1) / slices;
  const int64_t used = (nunits + ups - 1) / ups;
  if (groups > 0x7fffffff) return hipErrorInvalidValue;
  auto* kern = ((a.npix | b.npix) & 3) == 0 ? k_u8_to_bits<true> : k_u8_to_bits<false>;
  hipLaunchKernelGGL(kern, dim3(unsigned(groups), unsigned(used)), dim3(256), 0, s, a, b, groups0,
                     n, kpad_bits / 32, nunits, ups, stats);
  return hipGetLastError();
}

hipError_t u8_to_bytes(const IngestJob& a, const IngestJob& b, int64_t n, int64_t kpad_bytes,
                       const uint32_t* stats, hipStream_t s) {
  const int64_t fblocks = kpad_bytes / 64;
  const int64_t tiles_p0 = a.npix_pad / 64, tiles_p1 = b.npix_pad / 64;
  const int64_t tiles0 = tiles_p0 * fblocks;
  const int64_t tiles = tiles0 + tiles_p1 * fblocks;
  const int64_t grid = tiles < 4096 ? tiles : 4096;
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL(k_u8_to_bytes, dim3(unsigned(grid)), dim3(256), 0, s, a, b, n, kpad_bytes,
                     tiles_p0, tiles0, tiles_p1, tiles, stats);
  return hipGetLastError();
}

hipError_t split_sidebyside(const uint8_t* frames, int64_t n, int frame_w, int frame_h, int roi_x,
                            int roi_y, int roi_w, int roi_h, uint8_t* out_a, uint8_t* out_b,
                            hipStream_t s) {
  const int64_t in_fbytes = (int64_t(frame_w) * frame_h + 7) / 8;
  const int64_t out_fbytes = (int64_t(roi_w) * roi_h + 7) / 8;
  const int64_t total = 2 * n * out_fbytes;
  hipLaunchKernelGGL(k_split_sbs, dim3(grid_for(total, 256)), dim3(256), 0, s, frames, n,
                     in_fbytes, frame_w, roi_x, roi_y, roi_w, roi_h, out_a, out_b, out_fbytes);
  return hipGetLastError();
}

}  // namespace cpi
