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

// In-place transpose of a 32 x 32 bit block: on entry bit j of d[k] is
// element (k, j), on return bit k of d[j] is that element.  Five rounds of
// block exchanges (Hacker's Delight, section 7-3, in least-significant-bit-
// first order): round s swaps the upper s bits of each 2s-bit group of row k
// with the lower s bits of the same group of row k + s, for every k with bit
// s clear.
__host__ __device__ __forceinline__ void transpose32(uint32_t (&d)[32]) {
  constexpr uint32_t mask[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const int s = 16 >> r;
    const uint32_t m = mask[r];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (k & s) continue;
      const uint32_t t = ((d[k] >> s) ^ d[k + s]) & m;
      d[k] ^= t << s;
      d[k + s] ^= t;
    }
  }
}

constexpr int kBitsTilePix = 1024;   // pixels per work-group tile (32 words of a frame row)
constexpr int kBitsTileFr = 512;     // frames per tile (16 words of a bit row)
// The tile is staged frame word by frame word: word fw of pixel 32 q + i at
// stage[fw * kBitsLdsCol + 32 i + q].  The column stride (1060 = 36 mod 64)
// keeps the two half-waves' writes (adjacent frame words) and the row-segment
// reads (four frame words 4 apart) on distinct banks, and every offset of a
// lane's accesses is an instruction immediate.
constexpr int kBitsLdsCol = 1060;

// Packed-bit frames -> bit rows, for the 512-frame tiles that lie wholly
// below n, when frame rows are a multiple of 4 bytes long (k_ingest_bits_tail
// writes the rest).  A work-group (4 waves) owns 1024 pixels and a slice of
// those tiles.  For each tile, each half-wave takes 32
// frames: lane q of the half reads word q of the tile's row segment in each
// of the 32 frames (a half reads 128 contiguous bytes per frame) and
// transposes the 32 x 32 bit block in registers, which leaves it the 32
// frame bits of pixels 32 q .. 32 q + 31.  The words go to LDS and are
// written out as 64-byte row segments (four lanes per row, 16 bytes each).  Per-pixel popcounts are kept in registers,
// combined in LDS, and added to sums once per work-group.
__global__ __launch_bounds__(256, 2) void k_ingest_bits(IngestJob j0, IngestJob j1, int64_t groups0,
                                                    int64_t n, int64_t kw, int64_t ntiles,
                                                    int64_t tiles_per_slice) {
  __shared__ uint32_t stage[16 * kBitsLdsCol];
  __shared__ uint32_t psum[kBitsTilePix];
  // work-groups [0, groups0) take detector job j0, the rest job j1
  const bool second = int64_t(blockIdx.x) >= groups0;
  const IngestJob& job = second ? j1 : j0;
  const uint8_t* __restrict__ frames = job.frames;
  const int64_t fbytes = (job.npix + 7) / 8;
  const int64_t npix_pad = job.npix_pad;
  uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(job.out);
  const int swap02 = job.swap02;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int q = lane & 31, half = lane >> 5;
  const int64_t p0 = (int64_t(blockIdx.x) - (second ? groups0 : 0)) * kBitsTilePix;
  const int64_t byte = p0 / 8 + 4 * q;   // this lane's word in every frame row
  const int64_t kt0 = int64_t(blockIdx.y) * tiles_per_slice;
  int64_t kt1 = kt0 + tiles_per_slice;
  if (kt1 > ntiles) kt1 = ntiles;

  for (int i = tid; i < kBitsTilePix; i += 256) psum[i] = 0u;
  uint32_t cnt[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) cnt[i] = 0u;

  // The two 32-frame blocks of this lane in tile kt: frame words 2 wave +
  // half and 8 + 2 wave + half of the tile (every frame of the tile is below
  // n).  Buffer loads whose descriptor starts at the tile's first frame: the
  // lane's row offset (block and byte) is the vector offset and the frame's
  // row offset within the block the scalar one, so that no per-load address
  // registers are needed.  Words past a frame row reread the row's first
  // word and are masked to zero.  (Offsets stay below 2^31: rows are under
  // 2^22 bytes.)
  const bool word_in = byte + 4 <= fbytes;
  const uint32_t word_mask = word_in ? 0xffffffffu : 0u;
  int voff[2];
#pragma unroll
  for (int pass = 0; pass < 2; ++pass)
    voff[pass] = int((8 * pass + 2 * wave + half) * 32 * fbytes + (word_in ? byte : 0));
  auto load_tile = [&](int64_t kt, uint32_t(&d)[2][32]) {
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(frames + kt * kBitsTileFr * fbytes), short(0), 0x7fffffff,
        0x00020000);
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int k = 0; k < 32; ++k)
        d[pass][k] =
            uint32_t(__builtin_amdgcn_raw_buffer_load_b32(rb, voff[pass], int(k * fbytes), 0)) &
            word_mask;
  };
  // row-segment writes: lane 4 r + e writes words 4 e .. 4 e + 3 of row
  // 32 q2 + 2 j + wave / 2 (q2 = r + 16 (wave & 1)) for j = 0 .. 15
  const int q2 = (lane >> 2) + 16 * (wave & 1), c2 = 4 * (lane & 3);
  const int64_t row2 = p0 + 32 * q2 + (wave >> 1);
  const int vo2 = int(((32 * q2 + (wave >> 1)) * kw + c2) * 4);
  const __amdgpu_buffer_rsrc_t ors = __builtin_amdgcn_make_buffer_rsrc(
      out + p0 * kw, short(0), 0x7fffffff, 0x00020000);
  uint32_t cur[2][32], nxt[2][32];
  if (kt0 < kt1) load_tile(kt0, cur);
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    // the next tile's loads are in flight while this one is transposed and
    // written (straight-line: the last tile loads itself again)
    load_tile(kt + 1 < kt1 ? kt + 1 : kt, nxt);
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int fw = 8 * pass + 2 * wave + half;
      transpose32(cur[pass]);
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        cnt[i] += __popc(cur[pass][i]);
        const uint32_t w = swap02 ? swap_bits02(cur[pass][i]) : cur[pass][i];
        stage[fw * kBitsLdsCol + 32 * i + q] = w;
      }
    }
    __syncthreads();
    // 1024 rows x 16 words, 16 bytes per lane: consecutive lanes cover one
    // 64-byte segment of a row.
    // (buffer stores: the lane's row and word are the vector offset, the
    // pass's row step and the tile's column the scalar one)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int i = 2 * j + (wave >> 1);
      const uint32_t* src = stage + c2 * kBitsLdsCol + 32 * i + q2;
      typedef uint32_t u4v __attribute__((ext_vector_type(4)));
      const u4v v = {src[0], src[kBitsLdsCol], src[2 * kBitsLdsCol], src[3 * kBitsLdsCol]};
      if (row2 + 2 * j < npix_pad)
        __builtin_amdgcn_raw_buffer_store_b128(v, ors, vo2, int((2 * j * kw + kt * 16) * 4), 0);
    }
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int k = 0; k < 32; ++k) cur[pass][k] = nxt[pass][k];
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) atomicAdd(&psum[32 * q + i], cnt[i]);
  __syncthreads();
  unsigned long long* __restrict__ sums = reinterpret_cast<unsigned long long*>(job.sums);
  for (int i = tid; i < kBitsTilePix; i += 256)
    if (p0 + i < npix_pad) atomicAdd(&sums[p0 + i], (unsigned long long)psum[i]);
}

// Packed-bit frames -> bit rows for row words [w0, kw) (frames 32 w0 ..):
// one thread per (pixel word q, row word w) of either detector (w fastest),
// which reads word q of frames 32 w .. 32 w + 31 (guarded word loads, or byte
// loads when rows are not whole words: bits of pixels at or past 8 * row
// bytes, and of frames at or past n, are zero)
// and transposes the 32 x 32 block into row word w of pixels 32 q .. 32 q + 31.
// Popcounts are combined per work-group in LDS, then added to sums.
__global__ __launch_bounds__(256) void k_ingest_bits_tail(IngestJob j0, IngestJob j1, int64_t n,
                                                         int64_t kw, int64_t w0) {
  constexpr int kRows = (256 + 2) * 32;   // rows a work-group can touch
  __shared__ uint32_t psum[kRows];
  const int64_t wt = kw - w0;   // row words per pixel word
  const int64_t q0a = j0.npix_pad / 32;
  const int64_t t0 = int64_t(blockIdx.x) * 256;
  const int64_t qlo = t0 / wt;   // first pixel word (over both detectors) of the block
  for (int i = threadIdx.x; i < kRows; i += 256) psum[i] = 0u;
  __syncthreads();
  const int64_t t = t0 + threadIdx.x;
  const int64_t qg = t / wt, w = w0 + t % wt;
  const bool second = qg >= q0a;
  const IngestJob& job = second ? j1 : j0;
  const int64_t q = second ? qg - q0a : qg;
  if (q < job.npix_pad / 32) {
    const int64_t fbytes = (job.npix + 7) / 8;
    uint32_t d[32];
    if ((fbytes & 3) == 0) {
      // whole-word rows: one 4-byte load per frame
      const bool win = 4 * q + 4 <= fbytes;
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const int64_t f = 32 * w + k;
        const bool ok = f < n && win;
        const uint32_t v = *reinterpret_cast<const uint32_t*>(
            job.frames + (ok ? f * fbytes + 4 * q : 0));
        d[k] = ok ? v : 0u;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const int64_t f = 32 * w + k;
        const uint8_t* row = job.frames + (f < n ? f : 0) * fbytes;
        uint32_t v = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int64_t by = 4 * q + b;
          const bool ok = f < n && by < fbytes;
          v |= (ok ? uint32_t(row[ok ? by : 0]) : 0u) << (8 * b);
        }
        d[k] = v;
      }
    }
    transpose32(d);
    uint32_t* __restrict__ out = reinterpret_cast<uint32_t*>(job.out) + 32 * q * kw + w;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      out[i * kw] = job.swap02 ? swap_bits02(d[i]) : d[i];
      if (d[i]) atomicAdd(&psum[(qg - qlo) * 32 + i], uint32_t(__popc(d[i])));
    }
  }
  __syncthreads();
  const int64_t qhi = (t0 + 255) / wt;
  for (int64_t r = threadIdx.x; r < (qhi - qlo + 1) * 32; r += 256) {
    const uint32_t c = psum[r];
    if (!c) continue;
    const int64_t qq = qlo + r / 32;
    const bool sec = qq >= q0a;
    const IngestJob& jb = sec ? j1 : j0;
    const int64_t p = (sec ? qq - q0a : qq) * 32 + r % 32;
    if (p < jb.npix_pad)
      atomicAdd(reinterpret_cast<unsigned long long*>(jb.sums) + p, (unsigned long long)c);
  }
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
  // a work-group of the tile kernel covers 1024 rows (the last one of a
  // detector may reach past npix_pad and writes only the rows below it) and
  // 512-frame tiles below n; the tail kernel writes the remaining words
  for (const IngestJob* j : {&a, &b})
    if (j->npix_pad % 128 != 0 || j->npix_pad < j->npix ||
        (j->npix + 7) / 8 >= (int64_t(1) << 22))
      return hipErrorInvalidValue;
  // (row offsets within a 1024-row tile stay below 2^31 bytes)
  if (kpad_bits % kBitsTileFr != 0 || n > kpad_bits || kpad_bits / 32 >= (int64_t(1) << 19))
    return hipErrorInvalidValue;
  const bool aligned = (((a.npix + 7) / 8) & 3) == 0 && (((b.npix + 7) / 8) & 3) == 0;
  const int64_t full = aligned ? n / kBitsTileFr : 0;   // tiles for the tile kernel
  const int64_t groups0 = (a.npix_pad + kBitsTilePix - 1) / kBitsTilePix;
  const int64_t groups = groups0 + (b.npix_pad + kBitsTilePix - 1) / kBitsTilePix;
  if (groups > 0x7fffffff) return hipErrorInvalidValue;
  if (full > 0 && groups > 0) {
    const int64_t slices = slices_for(groups, full, 2048);
    const int64_t tps = (full + slices - 1) / slices;
    const int64_t used = (full + tps - 1) / tps;
    hipLaunchKernelGGL(k_ingest_bits, dim3(unsigned(groups), unsigned(used)), dim3(256), 0, s, a,
                       b, groups0, n, kpad_bits / 32, full, tps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t kw = kpad_bits / 32, w0 = full * (kBitsTileFr / 32);
  const int64_t threads = (a.npix_pad + b.npix_pad) / 32 * (kw - w0);
  if (threads > 0) {
    if ((threads + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ingest_bits_tail, dim3(unsigned((threads + 255) / 256)), dim3(256), 0, s,
                       a, b, n, kw, w0);
    return hipGetLastError();
  }
  return hipSuccess;
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
