// Finalisation of the accumulated image (Sect. 3.1: the device image is
// accumulated over all work and then handed back) and the image-wide FP64
// reductions (per-channel flux and maximum), plus small fill kernels.
//
// Additive modes hold J = sum E tau per channel until here; the
// absorption-equals-emission mode maps it to 1 - exp(-J).  Reductions are
// deterministic: fixed grid, per-block FP64 partials, one final block that
// sums the partials in block order.
#include <algorithm>

#include "spl_internal.h"

namespace spl {

namespace {

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

// Small device-to-host read-back: one workgroup copies 32-bit words into
// page-locked host memory mapped into the device's address space.  Kept off
// the copy engines, so it never queues behind a large host-to-device copy on
// another stream.  With a completion word (flag): every lane makes its own
// copied words visible at system scope, then, after the workgroup barrier,
// lane 0 stores seq into flag, so a host that sees seq there also sees the
// words.
__global__ __launch_bounds__(kBlock) void k_readback(const uint32_t *__restrict__ src,
                                                     uint32_t *__restrict__ dst, int words,
                                                     uint32_t *flag, uint32_t seq) {
  for (int i = threadIdx.x; i < words; i += kBlock) dst[i] = src[i];
  if (!flag) return;
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_fill_f64(double *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_fill_f32(float *p, float v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

// Clears the images of several views (view blockIdx.y).
__global__ __launch_bounds__(kBlock) void k_clear_views(ImgViews iv) {
  float *const p = iv.img[blockIdx.y];
  const int64_t n = 3 * iv.n_px[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = 0.0f;
}

// Per block: FP64 sums of the final image (3), maxima (3) and sums of the
// values before the map (3: the additive J), in that order.  View
// v = blockIdx.y takes iv.blocks[v] blocks (the rest of its row of the grid
// exits), its partials at partials0 + v pstride.
__global__ __launch_bounds__(kBlock) void k_finalise(ImgViews iv, double *__restrict__ partials0,
                                                     size_t pstride) {
  __shared__ double s_red[kStatPartials][kBlock];
  const int v = blockIdx.y, nblk = iv.blocks[v];
  if ((int)blockIdx.x >= nblk) return;  // uniform
  float *__restrict__ img = iv.img[v];
  const int64_t n_px = iv.n_px[v];
  const int aeqe = iv.aeqe[v];
  double *__restrict__ partials = partials0 + v * pstride;
  double sm[3] = {0.0, 0.0, 0.0}, raw[3] = {0.0, 0.0, 0.0};
  double mx[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < n_px;
       p += (int64_t)nblk * kBlock) {
    float *o = img + 3 * p;
    float v[3] = {o[0], o[1], o[2]};
#pragma unroll
    for (int c = 0; c < 3; ++c) raw[c] += (double)v[c];
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
    s_red[6 + c][threadIdx.x] = raw[c];
  }
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_red[c][threadIdx.x] += s_red[c][threadIdx.x + d];
        s_red[3 + c][threadIdx.x] = fmax(s_red[3 + c][threadIdx.x], s_red[3 + c][threadIdx.x + d]);
        s_red[6 + c][threadIdx.x] += s_red[6 + c][threadIdx.x + d];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < kStatPartials)
    partials[kStatPartials * blockIdx.x + threadIdx.x] = s_red[threadIdx.x][0];
}

// stats[0..2] = flux, [3..5] = max per channel, [6] = max over channels,
// [7..9] = flux before the map; block partials summed in block order.  One
// workgroup per view v = blockIdx.x (partials at partials0 + v pstride,
// iv.blocks[v] of them; stats at stats0 + v sstride).
__global__ __launch_bounds__(kBlock) void k_reduce_stats(const double *__restrict__ partials0,
                                                         size_t pstride, ImgViews iv,
                                                         double *__restrict__ stats0,
                                                         size_t sstride) {
  __shared__ double s_red[kStatPartials][kBlock];
  const double *__restrict__ partials = partials0 + blockIdx.x * pstride;
  const int n_blocks = iv.blocks[blockIdx.x];
  double *__restrict__ stats = stats0 + blockIdx.x * sstride;
  double sm[3] = {0.0, 0.0, 0.0}, raw[3] = {0.0, 0.0, 0.0};
  double mx[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
  for (int b = threadIdx.x; b < n_blocks; b += kBlock) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sm[c] += partials[kStatPartials * b + c];
      mx[c] = fmax(mx[c], partials[kStatPartials * b + 3 + c]);
      raw[c] += partials[kStatPartials * b + 6 + c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s_red[c][threadIdx.x] = sm[c];
    s_red[3 + c][threadIdx.x] = mx[c];
    s_red[6 + c][threadIdx.x] = raw[c];
  }
  __syncthreads();
  for (int d = kBlock / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s_red[c][threadIdx.x] += s_red[c][threadIdx.x + d];
        s_red[3 + c][threadIdx.x] = fmax(s_red[3 + c][threadIdx.x], s_red[3 + c][threadIdx.x + d]);
        s_red[6 + c][threadIdx.x] += s_red[6 + c][threadIdx.x + d];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) stats[threadIdx.x] = s_red[threadIdx.x][0];
  if (threadIdx.x == 0) stats[6] = fmax(fmax(s_red[3][0], s_red[4][0]), s_red[5][0]);
  if (threadIdx.x >= 6 && threadIdx.x < 9) stats[threadIdx.x + 1] = s_red[threadIdx.x][0];
}

// Expected flux (a conservation check independent of the tile lists and the
// splat): for every active record, kappa = the sum of exp(-d^2/sigma^2) over
// the pixels of its box whose centres lie within the truncation radius, in
// FP64 from the record's screen position and width; the particle adds A x
// kappa per channel, A = E/(pi sigma^2) being the record's premultiplied
// colour, so the total is sum_p E_p kappa_p.  Only particles whose span
// marks them active count (the projection leaves the records of inactive
// particles unwritten).  One wave per particle at a time, its lanes striding
// over the box; FP64 partial sums per block.
__global__ __launch_bounds__(kBlock) void k_expected_flux(const float4 *__restrict__ rec,
                                                          const uint2 *__restrict__ span,
                                                          int64_t n, int W, int H, float nu,
                                                          double *__restrict__ partials) {
  __shared__ double s_red[3][kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / 64);
  double acc[3] = {0.0, 0.0, 0.0};  // lane 0's running sums
  for (int64_t k = (int64_t)blockIdx.x * (kBlock / 64) + wave; k < n; k += wstride) {
    if (span[k].x == kInactive) continue;
    const float4 r0 = rec[2 * k], r1 = rec[2 * k + 1];
    int i0, i1, j0, j1;
    if (!record_box(r0.x, r0.y, r0.z, r0.w, r1.x, nu, W, H, i0, i1, j0, j1)) continue;
    const double X = (double)r0.x + (double)r0.y, Y = (double)r0.z + (double)r0.w;
    const double sg = (double)r1.x, R = (double)nu * sg;
    const double R2 = R * R, inv_s2 = 1.0 / (sg * sg);
    const int64_t bw = i1 - i0 + 1, total = bw * (int64_t)(j1 - j0 + 1);
    double kappa = 0.0;
    for (int64_t t = lane; t < total; t += 64) {
      const int i = i0 + (int)(t % bw), j = j0 + (int)(t / bw);
      const double dx = (double)i + 0.5 - X, dy = (double)j + 0.5 - Y;
      const double d2 = dx * dx + dy * dy;
      if (d2 <= R2) kappa += exp(-d2 * inv_s2);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) kappa += __shfl_xor(kappa, o);
    if (lane == 0) {
      acc[0] += (double)r1.y * kappa;
      acc[1] += (double)r1.z * kappa;
      acc[2] += (double)r1.w * kappa;
    }
  }
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 3; ++c) s_red[c][wave] = acc[c];
  __syncthreads();
  if (threadIdx.x < 3) {
    double v = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) v += s_red[threadIdx.x][w];
    partials[3 * blockIdx.x + threadIdx.x] = v;
  }
}

// out[0..2] = sum of the blocks' expected-flux partials, in block order.
__global__ void k_reduce_expected(const double *__restrict__ partials, int n_blocks,
                                  double *__restrict__ out) {
  if (threadIdx.x < 3) {
    double v = 0.0;
    for (int b = 0; b < n_blocks; ++b) v += partials[3 * b + threadIdx.x];
    out[threadIdx.x] = v;
  }
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

hipError_t launch_readback(const void *src, void *dst_mapped, size_t bytes, hipStream_t s,
                           void *flag_mapped, uint32_t seq) {
  if (bytes == 0 && !flag_mapped) return hipSuccess;
  hipLaunchKernelGGL(k_readback, dim3(1), dim3(kBlock), 0, s, static_cast<const uint32_t *>(src),
                     static_cast<uint32_t *>(dst_mapped), (int)(bytes / 4),
                     static_cast<uint32_t *>(flag_mapped), seq);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n / 4 + 1, 4096)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_clear_views(const ImgViews &iv, int n_views, hipStream_t s) {
  if (n_views < 1 || n_views > kMaxLaunchViews) return hipErrorInvalidValue;
  int64_t mx = 0;
  for (int v = 0; v < n_views; ++v) mx = std::max(mx, 3 * iv.n_px[v]);
  hipLaunchKernelGGL(k_clear_views, dim3(blocks_for(mx / 4 + 1, 4096), n_views), dim3(kBlock), 0,
                     s, iv);
  return hipGetLastError();
}

hipError_t launch_finalise_views(const ImgViews &iv, int n_views, double *partials,
                                 size_t pstride, hipStream_t s) {
  if (n_views < 1 || n_views > kMaxLaunchViews) return hipErrorInvalidValue;
  int mx = 1;
  for (int v = 0; v < n_views; ++v) mx = std::max(mx, iv.blocks[v]);
  hipLaunchKernelGGL(k_finalise, dim3(mx, n_views), dim3(kBlock), 0, s, iv, partials, pstride);
  return hipGetLastError();
}

hipError_t launch_reduce_stats_views(const double *partials, size_t pstride, const ImgViews &iv,
                                     int n_views, double *stats, size_t sstride, hipStream_t s) {
  if (n_views < 1 || n_views > kMaxLaunchViews) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_stats, dim3(n_views), dim3(kBlock), 0, s, partials, pstride, iv,
                     stats, sstride);
  return hipGetLastError();
}

hipError_t launch_finalise(float *img, int64_t n_px, int aeqe, double *partials, int n_blocks,
                           hipStream_t s) {
  ImgViews iv;
  iv.img[0] = img;
  iv.n_px[0] = n_px;
  iv.blocks[0] = n_blocks;
  iv.aeqe[0] = aeqe;
  return launch_finalise_views(iv, 1, partials, 0, s);
}

hipError_t launch_reduce_stats(const double *partials, int n_blocks, double *stats,
                               hipStream_t s) {
  ImgViews iv;
  iv.blocks[0] = n_blocks;
  return launch_reduce_stats_views(partials, 0, iv, 1, stats, 0, s);
}

hipError_t launch_expected_flux(const float *rec, const uint2 *span, int64_t n, int W, int H,
                                float nu, double *partials, int n_blocks, double *out,
                                hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_expected_flux, dim3(n_blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<const float4 *>(rec), span, n, W, H, nu, partials);
  else
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, partials, 3 * n_blocks);
  hipLaunchKernelGGL(k_reduce_expected, dim3(1), dim3(64), 0, s, partials, n_blocks, out);
  return hipGetLastError();
}

hipError_t launch_normalise(float *img, int64_t n_px, const double *stats, hipStream_t s) {
  const int64_t n = 3 * n_px;
  hipLaunchKernelGGL(k_normalise, dim3(blocks_for(n, 4096)), dim3(kBlock), 0, s, img, n, stats);
  return hipGetLastError();
}

}  // namespace spl
