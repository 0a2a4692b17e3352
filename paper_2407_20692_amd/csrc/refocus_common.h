// Definitions shared by the refocus kernels: integer geometry, the clamped
// interpolation cell, the per-plane row table entry and a vector-memory wait.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cpi {
namespace {

struct GeomI {
  int wa, ha, wb, hb, out_w, out_h;
};

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

// Row table of one plane: for output row y_r and lens-plane row y_b, the
// clamped interpolation row and its two weights (the arithmetic of the
// column side), laid out [plane][y_b][y_r] so that a wave's consecutive
// output rows are one scalar load.
struct YEntry {
  int row;
  float w0, w1;
  int pad;
};

// Wait until at most N vector-memory operations of this wave are in flight.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

}  // namespace
}  // namespace cpi
