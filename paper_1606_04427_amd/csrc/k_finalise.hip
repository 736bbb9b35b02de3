// Finalisation of the accumulated image (Sect. 3.1: the device image is
// accumulated over all work and then handed back) and the image-wide FP64
// reductions (per-channel flux and maximum), plus small fill kernels.
//
// Additive modes hold J = sum E tau per channel until here; the
// absorption-equals-emission mode maps it to 1 - exp(-J).  Reductions are
// deterministic: fixed grid, per-block FP64 partials, one final block that
// sums the partials in block order.
#include "spl_internal.h"

namespace spl {

namespace {

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_f32(float *p, float v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_finalise(float *__restrict__ img, int64_t n_px,
                                                     int aeqe, double *__restrict__ partials) {
  __shared__ double s_red[6][kBlock];
  double sm[3] = {0.0, 0.0, 0.0};
  double mx[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n_px;
       p += (int64_t)gridDim.x * kBlock) {
    float *o = img + 3 * p;
    float v[3] = {o[0], o[1], o[2]};
    if (aeqe) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[c] = -expm1f(-v[c]);
        o[c] = v[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sm[c] += (double)v[c];
      mx[c] = fmax(mx[c], (double)v[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s_red[c][threadIdx.x] = sm[c];
    s_red[3 + c][threadIdx.x] = mx[c];
  }
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_red[c][threadIdx.x] += s_red[c][threadIdx.x + d];
        s_red[3 + c][threadIdx.x] = fmax(s_red[3 + c][threadIdx.x], s_red[3 + c][threadIdx.x + d]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) partials[6 * blockIdx.x + threadIdx.x] = s_red[threadIdx.x][0];
}

// stats[0..2] = flux, [3..5] = max per channel, [6] = max over channels.
__global__ __launch_bounds__(kBlock) void k_reduce_stats(const double *__restrict__ partials,
                                                         int n_blocks, double *__restrict__ stats) {
  __shared__ double s_red[6][kBlock];
  double sm[3] = {0.0, 0.0, 0.0};
  double mx[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
  for (int b = threadIdx.x; b < n_blocks; b += kBlock) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sm[c] += partials[6 * b + c];
      mx[c] = fmax(mx[c], partials[6 * b + 3 + c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s_red[c][threadIdx.x] = sm[c];
    s_red[3 + c][threadIdx.x] = mx[c];
  }
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_red[c][threadIdx.x] += s_red[c][threadIdx.x + d];
        s_red[3 + c][threadIdx.x] = fmax(s_red[3 + c][threadIdx.x], s_red[3 + c][threadIdx.x + d]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) stats[threadIdx.x] = s_red[threadIdx.x][0];
  if (threadIdx.x == 0) stats[6] = fmax(fmax(s_red[3][0], s_red[4][0]), s_red[5][0]);
}

__global__ __launch_bounds__(kBlock) void k_normalise(float *__restrict__ img, int64_t n,
                                                      const double *__restrict__ stats) {
  const double m = stats[6];
  if (!(m > 0.0)) return;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    img[i] = (float)((double)img[i] / m);
}

int blocks_for(int64_t n, int cap) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 2048)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n / 4 + 1, 4096)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_finalise(float *img, int64_t n_px, int aeqe, double *partials, int n_blocks,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalise, dim3(n_blocks), dim3(kBlock), 0, s, img, n_px, aeqe, partials);
  return hipGetLastError();
}

hipError_t launch_reduce_stats(const double *partials, int n_blocks, double *stats,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(kBlock), 0, s, partials, n_blocks, stats);
  return hipGetLastError();
}

hipError_t launch_normalise(float *img, int64_t n_px, const double *stats, hipStream_t s) {
  const int64_t n = 3 * n_px;
  hipLaunchKernelGGL(k_normalise, dim3(blocks_for(n, 4096)), dim3(kBlock), 0, s, img, n, stats);
  return hipGetLastError();
}

}  // namespace spl
