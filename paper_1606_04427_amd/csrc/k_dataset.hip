// Conversion of particle attributes to the stored format of a resident data
// set (Sect. 2.1: data sets are converted to the code's internal format as
// they are read).  Stored attributes are FP32, BF16 or FP16; FP16 values
// carry a power-of-two scale per array that puts the largest finite
// magnitude near 2^10, so small smoothing lengths stay normal numbers.
//
// k_absmax   largest finite |v| of an array (the FP16 scale's input)
// k_convert  v = source value x source scale, stored as v / scale in the
//            stored type, rounded to nearest even
#include "spl_internal.h"

namespace spl {

namespace {

__device__ __forceinline__ float load_value(const void *p, int dtype, int64_t i) {
  if (dtype == SPL_F32) return static_cast<const float *>(p)[i];
  if (dtype == SPL_BF16) {
    const uint32_t b = static_cast<const uint16_t *>(p)[i];
    return __uint_as_float(b << 16);
  }
  return (float)static_cast<const _Float16 *>(p)[i];
}

// FP32 -> BF16, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t to_bf16(float v) {
  const uint32_t u = __float_as_uint(v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(kBlock) void k_absmax(const void *__restrict__ src, int dtype,
                                                   float scale, int64_t n,
                                                   uint32_t *__restrict__ out_bits) {
  __shared__ uint32_t s_m;
  if (threadIdx.x == 0) s_m = 0u;
  __syncthreads();
  uint32_t m = 0u;  // bits of a non-negative float order like the float
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const float v = fabsf(load_value(src, dtype, i) * scale);
    if (__builtin_isfinite(v)) m = max(m, __float_as_uint(v));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  if ((threadIdx.x & 63) == 0 && m) atomicMax(&s_m, m);
  __syncthreads();
  if (threadIdx.x == 0 && s_m) atomicMax(out_bits, s_m);
}

__global__ __launch_bounds__(kBlock) void k_convert(const void *__restrict__ src, int sdtype,
                                                    float sscale, void *__restrict__ dst,
                                                    int ddtype, float inv_dscale, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const float v = load_value(src, sdtype, i) * sscale * inv_dscale;
    if (ddtype == SPL_F32)
      static_cast<float *>(dst)[i] = v;
    else if (ddtype == SPL_BF16)
      static_cast<uint16_t *>(dst)[i] = to_bf16(v);
    else
      static_cast<_Float16 *>(dst)[i] = (_Float16)v;
  }
}

int grid_of(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (int)g;
}

}  // namespace

hipError_t launch_absmax(const void *src, int dtype, float scale, int64_t n, uint32_t *out_bits,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_absmax, dim3(grid_of(n)), dim3(kBlock), 0, s, src, dtype, scale, n,
                     out_bits);
  return hipGetLastError();
}

hipError_t launch_convert(const void *src, int sdtype, float sscale, void *dst, int ddtype,
                          float inv_dscale, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert, dim3(grid_of(n)), dim3(kBlock), 0, s, src, sdtype, sscale, dst,
                     ddtype, inv_dscale, n);
  return hipGetLastError();
}

}  // namespace spl
