// Reference kernels for the rooflines (not part of the method): a plain
// device copy, whose duration gives the attainable HBM bandwidth and whose
// hardware-counter readings calibrate the traffic counters of the other
// kernels, and an MFMA issue loop per precision, whose rate gives the
// attainable matrix-core throughput at the clock the chip holds under load.
#include "ls_split_tile.hpp"

namespace ls {

// Each workgroup copies one contiguous block of 1024 16-byte elements: four
// independent loads per thread, all issued before the stores.
__global__ __launch_bounds__(256) void k_probe_copy(const uint4* __restrict__ src,
                                                     uint4* __restrict__ dst, size_t n) {
  const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
  uint4 v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (base + 256 * e < n) v[e] = src[base + 256 * e];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (base + 256 * e < n) dst[base + 256 * e] = v[e];
}

// Each wave keeps 8 (16x16 shapes) or 4 (32x32 shapes) independent
// accumulators so that the issue of one MFMA never waits for the result of
// the previous one.
typedef float f16v_probe_t __attribute__((ext_vector_type(16)));

template <int P, int SHAPE>
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  float r = 0.0f;
  if constexpr (SHAPE == 1 && P == LS_F32) {
    const float x = 1.0f + 1e-3f * lane, z = 0.5f - 1e-4f * lane;
    f16v_probe_t acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[u][v] = 0.0f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, z, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 16; ++v) r += acc[u][v];
  } else if constexpr (SHAPE == 1 && P == LS_F16X3) {
    h8_t x, z;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      x[e] = (_Float16)(1.0f + 0.125f * ((lane + e) & 7));
      z[e] = (_Float16)(0.5f + 0.125f * ((lane * 3 + e) & 7));
    }
    f16v_probe_t acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[u][v] = 0.0f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_f16(x, z, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 16; ++v) r += acc[u][v];
  } else if constexpr (SHAPE == 1) {
    s8_t xs, zs;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      xs[e] = (short)(0x3f80 + ((lane + e) & 7));
      zs[e] = (short)(0x3f00 + ((lane * 3 + e) & 7));
    }
    const bf8_t x = __builtin_bit_cast(bf8_t, xs), z = __builtin_bit_cast(bf8_t, zs);
    f16v_probe_t acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[u][v] = 0.0f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, z, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 16; ++v) r += acc[u][v];
  } else if constexpr (P == LS_F64) {
    const double x = 1.0 + 1e-3 * lane, z = 0.5 - 1e-4 * lane;
    d4_t acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = d4_t{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, z, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 8; ++u) r += (float)(acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3]);
  } else if constexpr (P == LS_F32) {
    const float x = 1.0f + 1e-3f * lane, z = 0.5f - 1e-4f * lane;
    f4_t acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = f4_t{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, z, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 8; ++u) r += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  } else if constexpr (P == LS_F16X3) {
    h8_t x, z;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      x[e] = (_Float16)(1.0f + 0.125f * ((lane + e) & 7));
      z[e] = (_Float16)(0.5f + 0.125f * ((lane * 3 + e) & 7));
    }
    f4_t acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = f4_t{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, z, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 8; ++u) r += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  } else {
    s8_t xs, zs;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      xs[e] = (short)(0x3f80 + ((lane + e) & 7));  // bf16 values near 1
      zs[e] = (short)(0x3f00 + ((lane * 3 + e) & 7));
    }
    const bf8_t x = __builtin_bit_cast(bf8_t, xs), z = __builtin_bit_cast(bf8_t, zs);
    f4_t acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = f4_t{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, z, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 8; ++u) r += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  }
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;
}

}  // namespace ls

using namespace ls;

extern "C" ls_status ls_probe_copy(const void* src_dev, void* dst_dev, size_t bytes,
                                   hipStream_t stream) {
  clear_error();
  LS_REQUIRE(src_dev != nullptr && dst_dev != nullptr, "null device pointer");
  LS_REQUIRE(bytes % 16 == 0 && bytes > 0, "bytes must be a positive multiple of 16");
  LS_REQUIRE(((uintptr_t)src_dev | (uintptr_t)dst_dev) % 16 == 0, "pointers must be 16-byte aligned");
  const size_t n = bytes / 16;
  const size_t blocks = (n + 1023) / 1024;
  LS_REQUIRE(blocks <= 0x7fffffff, "copy too large");
  hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)blocks), dim3(256), 0, stream,
                     (const uint4*)src_dev, (uint4*)dst_dev, n);
  return launch_status("ls_probe_copy");
}

extern "C" ls_status ls_probe_mfma(int32_t precision, int32_t shape, int32_t blocks, int32_t iters,
                                   float* out_dev, double* flops, hipStream_t stream) {
  clear_error();
  LS_REQUIRE(out_dev != nullptr && flops != nullptr, "null pointer");
  LS_REQUIRE(blocks >= 1 && blocks <= (1 << 20), "blocks must be in [1, 2^20]");
  LS_REQUIRE(iters >= 1 && iters <= (1 << 24), "iters must be in [1, 2^24]");
  LS_REQUIRE(shape == 0 || shape == 1, "shape must be 0 (16x16) or 1 (32x32)");
  LS_REQUIRE(!(shape == 1 && precision == LS_F64), "no 32x32 FP64 instruction");
  double per = 0.0;  // flops per wave per loop iteration
  const dim3 g(blocks), b(256);
  switch (precision) {
    case LS_F64:
      hipLaunchKernelGGL((k_probe_mfma<LS_F64, 0>), g, b, 0, stream, iters, out_dev);
      per = 8 * 2.0 * 16 * 16 * 4;
      break;
    case LS_F32:
      if (shape == 0) {
        hipLaunchKernelGGL((k_probe_mfma<LS_F32, 0>), g, b, 0, stream, iters, out_dev);
        per = 8 * 2.0 * 16 * 16 * 4;
      } else {
        hipLaunchKernelGGL((k_probe_mfma<LS_F32, 1>), g, b, 0, stream, iters, out_dev);
        per = 4 * 2.0 * 32 * 32 * 2;
      }
      break;
    case LS_BF16X3:
    case LS_BF16X6:
      if (shape == 0) {
        hipLaunchKernelGGL((k_probe_mfma<LS_BF16X3, 0>), g, b, 0, stream, iters, out_dev);
        per = 8 * 2.0 * 16 * 16 * 32;
      } else {
        hipLaunchKernelGGL((k_probe_mfma<LS_BF16X3, 1>), g, b, 0, stream, iters, out_dev);
        per = 4 * 2.0 * 32 * 32 * 16;
      }
      break;
    case LS_F16X3:
      if (shape == 0) {
        hipLaunchKernelGGL((k_probe_mfma<LS_F16X3, 0>), g, b, 0, stream, iters, out_dev);
        per = 8 * 2.0 * 16 * 16 * 32;
      } else {
        hipLaunchKernelGGL((k_probe_mfma<LS_F16X3, 1>), g, b, 0, stream, iters, out_dev);
        per = 4 * 2.0 * 32 * 32 * 16;
      }
      break;
    default:
      set_error("unknown precision %d", precision);
      return LS_EINVAL;
  }
  *flops = per * iters * 4.0 * blocks;
  return launch_status("ls_probe_mfma");
}
