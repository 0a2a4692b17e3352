// Measured peaks of this device: register-only loops of the two matrix-core
// ops the contraction uses (int8 16x16x64 and FP4 16x16x128 with FP32 sums)
// and a streaming device copy.  They put the vendor figures the rooflines are
// quoted against next to what the part sustains.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpi {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kLoopIters = 400;

// 16 independent accumulators per wave; operands are binary-like data (about
// one bit in ten set), as in the contraction.
template <bool FP4>
__global__ __launch_bounds__(256) void k_mfma_loop(const uint32_t* __restrict__ in,
                                                   uint32_t* __restrict__ out) {
  const int t = threadIdx.x;
  const uint32_t x0 = in[t & 255], x1 = in[(t + 64) & 255];
  if constexpr (FP4) {
    v8i a[4], b[4];
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = v8i{int(x0 + i), int(x1), int(x0), int(x1 ^ i), 0, 0, 0, 0};
      b[i] = v8i{int(x1 + i), int(x0), int(x1), int(x0 ^ i), 0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0, 0, 0, 0};
    for (int it = 0; it < kLoopIters; ++it) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[i], b[j], acc[i][j], 4,
                                                                       4, 0, 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) s += acc[i][j][0] + acc[i][j][3];
    out[blockIdx.x * 256 + t] = uint32_t(s);
  } else {
    v4i a[4], b[4], acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = v4i{int(x0 + i), int(x1), int(x0), int(x1 ^ i)};
      b[i] = v4i{int(x1 + i), int(x0), int(x1), int(x0 ^ i)};
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};
    for (int it = 0; it < kLoopIters; ++it) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) s += acc[i][j][0] + acc[i][j][3];
    out[blockIdx.x * 256 + t] = uint32_t(s);
  }
}

__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * 256)
    dst[i] = src[i];
}

}  // namespace

size_t peaks_scratch_bytes(size_t copy_bytes) { return 2 * copy_bytes + 1024 + 2048 * 256 * 4; }

hipError_t measure_peaks(uint8_t* scratch, size_t copy_bytes, hipStream_t s, double* int8_ops,
                         double* fp4_ops, double* copy_bytes_per_s) {
  const int wgs = 2048;   // 8 work-groups of 4 waves per CU on 256 CUs
  uint32_t* in = reinterpret_cast<uint32_t*>(scratch);
  uint32_t* out = reinterpret_cast<uint32_t*>(scratch + 1024);
  uint8_t* cbuf = scratch + 1024 + size_t(wgs) * 256 * 4;
  hipError_t e;
  // operands: about one bit in ten set, like the frames
  uint32_t host[256];
  uint32_t st = 12345u;
  for (int i = 0; i < 256; ++i) {
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) {
      st = st * 1664525u + 1013904223u;
      if ((st >> 24) < 26u) v |= 1u << b;
    }
    host[i] = v & 0x22222222u;
  }
  if ((e = hipMemcpyAsync(in, host, sizeof(host), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  hipEvent_t e0, e1;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    hipEventDestroy(e0);
    return e;
  }
  auto timed = [&](auto launch, double work, double* rate) -> hipError_t {
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      hipEventRecord(e0, s);
      launch();
      hipEventRecord(e1, s);
      hipError_t r = hipEventSynchronize(e1);
      if (r != hipSuccess) return r;
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0 && ms < best) best = ms;   // the first run warms up
    }
    *rate = work / (double(best) * 1e-3);
    return hipGetLastError();
  };
  const double waves = double(wgs) * 4;
  e = timed([&] { hipLaunchKernelGGL(k_mfma_loop<false>, dim3(wgs), dim3(256), 0, s, in, out); },
            waves * kLoopIters * 16 * 2.0 * 16 * 16 * 64, int8_ops);
  if (e == hipSuccess)
    e = timed([&] { hipLaunchKernelGGL(k_mfma_loop<true>, dim3(wgs), dim3(256), 0, s, in, out); },
              waves * kLoopIters * 16 * 2.0 * 16 * 16 * 128, fp4_ops);
  if (e == hipSuccess) {
    const int64_t count = int64_t(copy_bytes / 16);
    const uint4* src = reinterpret_cast<const uint4*>(cbuf);
    uint4* dst = reinterpret_cast<uint4*>(cbuf + copy_bytes);
    e = timed([&] { hipLaunchKernelGGL(k_copy16, dim3(8192), dim3(256), 0, s, src, dst, count); },
              2.0 * double(count) * 16, copy_bytes_per_s);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return e;
}

}  // namespace cpi
