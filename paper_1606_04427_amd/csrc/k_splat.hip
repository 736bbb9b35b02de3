// Render stage (Sect. 3.1: each tile's list is rendered by one worker that
// owns the tile's pixels; Sect. 3.2.2: drawing adds colour x contribution to
// the pixel).  One workgroup per work item = one chunk of one tile's list;
// the tile's pixels live in registers and LDS, so no two workgroups share a
// pixel except the chunks of one long list, which merge by hardware float
// atomics (additive) or by an ordered merge of partial (colour,
// transmittance) tiles (sorted).
//
// k_splat_add<T>   additive modes, T x T tile, 256 lanes.  Each batch of 256
//                  list entries is loaded once, one entry per lane.  Entries
//                  whose box covers few of the tile's pixels are scattered by
//                  their own lane into an LDS accumulator with LDS float
//                  atomics; larger ones are staged in LDS and gathered by all
//                  lanes, one pixel per lane, skipping (wave-uniformly) the
//                  ones that miss a wave's rows.  After every batch the LDS
//                  and register partials are folded into per-pixel
//                  Neumaier-compensated sums.
// k_splat_large    the large-particle path: 64 x 64 px tiles, 512 lanes, 8
//                  pixels per lane, gather only (a large particle covers most
//                  of the pixels it is tested against).
// k_composite<T>   sorted mode: front-to-back slab compositing in list order,
//                  one pixel per lane (T = 16) or 4 (T = 32); transmittance
//                  per pixel in registers.
#include "spl_internal.h"

namespace spl {

namespace {

__device__ __forceinline__ void neumaier(float &sum, float &comp, float v) {
  const float t = sum + v;
  if (fabsf(sum) >= fabsf(v))
    comp += (sum - t) + v;
  else
    comp += (v - t) + sum;
  sum = t;
}

__device__ __forceinline__ uint32_t pack_box(int a0, int a1, int b0, int b1) {
  return (uint32_t)a0 | ((uint32_t)a1 << 8) | ((uint32_t)b0 << 16) | ((uint32_t)b1 << 24);
}

template <int T>
__global__ __launch_bounds__(kBlock) void k_splat_add(const Item *__restrict__ items,
                                                      const uint32_t *__restrict__ pairs,
                                                      const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ counts,
                                                      int chunk, TileK tk, int scat_max,
                                                      float *__restrict__ img) {
  constexpr int NP = T * T;
  constexpr int PX = NP / kBlock;
  constexpr int WROWS = (64 / T) * PX;  // rows covered by one wave
  __shared__ float acc[3 * NP];
  __shared__ float g_ox[kBlock], g_fx[kBlock], g_oy[kBlock], g_fy[kBlock], g_is2[kBlock];
  __shared__ float g_a0[kBlock], g_a1[kBlock], g_a2[kBlock];
  __shared__ uint32_t g_box[kBlock];
  __shared__ int g_count;

  const Item it = items[blockIdx.x];
  const int tx = (int)it.x % tk.ntx, ty = (int)it.x / tk.ntx;
  const int x0 = tx * T, y0 = ty * T;
  const bool multi = counts[it.x] > (uint32_t)chunk;
  const int tid = threadIdx.x;
  const int pc = tid % T;
  const int pr0 = (tid / T) * PX;
  const int wr0 = (tid / 64) * WROWS, wr1 = wr0 + WROWS - 1;
  const float nu2 = tk.nu * tk.nu;

  float sum[PX][3], comp[PX][3], bs[PX][3];
#pragma unroll
  for (int m = 0; m < PX; ++m)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sum[m][c] = 0.f;
      comp[m][c] = 0.f;
      bs[m][c] = 0.f;
    }
  for (int i = tid; i < 3 * NP; i += kBlock) acc[i] = 0.f;

  for (uint32_t base = it.y; base < it.z; base += kBlock) {
    if (tid == 0) g_count = 0;
    __syncthreads();
    const uint32_t k = base + tid;
    if (k < it.z) {
      const uint32_t pid = pairs[k];
      const float4 r0 = rec[2 * (size_t)pid];
      const float4 r1 = rec[2 * (size_t)pid + 1];
      int i0, i1, j0, j1;
      if (record_box(r0.x, r0.y, r0.z, r0.w, r1.x, tk.nu, tk.W, tk.H, i0, i1, j0, j1)) {
        const int li0 = max(i0 - x0, 0), li1 = min(i1 - x0, T - 1);
        const int lj0 = max(j0 - y0, 0), lj1 = min(j1 - y0, T - 1);
        if (li0 <= li1 && lj0 <= lj1) {
          const float ox = r0.x - (float)x0, fx = 0.5f - r0.y;
          const float oy = r0.z - (float)y0, fy = 0.5f - r0.w;
          const float is2 = 1.0f / (r1.x * r1.x);
          const int area = (li1 - li0 + 1) * (lj1 - lj0 + 1);
          if (area <= scat_max) {
            for (int jj = lj0; jj <= lj1; ++jj) {
              const float dy = ((float)jj - oy) + fy;
              for (int ii = li0; ii <= li1; ++ii) {
                const float dx = ((float)ii - ox) + fx;
                const float q = (dx * dx + dy * dy) * is2;
                if (q <= nu2) {
                  const float g = __expf(-q);
                  const int pix = jj * T + ii;
                  atomicAdd(&acc[pix], r1.y * g);
                  atomicAdd(&acc[NP + pix], r1.z * g);
                  atomicAdd(&acc[2 * NP + pix], r1.w * g);
                }
              }
            }
          } else {
            const int slot = atomicAdd(&g_count, 1);
            g_ox[slot] = ox;
            g_fx[slot] = fx;
            g_oy[slot] = oy;
            g_fy[slot] = fy;
            g_is2[slot] = is2;
            g_a0[slot] = r1.y;
            g_a1[slot] = r1.z;
            g_a2[slot] = r1.w;
            g_box[slot] = pack_box(li0, li1, lj0, lj1);
          }
        }
      }
    }
    __syncthreads();
    const int ng = g_count;
    for (int g = 0; g < ng; ++g) {
      const uint32_t bx = g_box[g];
      const int li0 = bx & 0xff, li1 = (bx >> 8) & 0xff, lj0 = (bx >> 16) & 0xff,
                lj1 = bx >> 24;
      if (lj1 < wr0 || lj0 > wr1) continue;  // uniform across the wave
      if (pc < li0 || pc > li1) continue;
      const float dx = ((float)pc - g_ox[g]) + g_fx[g];
      const float dx2 = dx * dx;
      const float is2 = g_is2[g], oy = g_oy[g], fy = g_fy[g];
#pragma unroll
      for (int m = 0; m < PX; ++m) {
        const int row = pr0 + m;
        if (row < lj0 || row > lj1) continue;
        const float dy = ((float)row - oy) + fy;
        const float q = (dx2 + dy * dy) * is2;
        if (q <= nu2) {
          const float e = __expf(-q);
          bs[m][0] += g_a0[g] * e;
          bs[m][1] += g_a1[g] * e;
          bs[m][2] += g_a2[g] * e;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PX; ++m) {
      const int pix = (pr0 + m) * T + pc;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float v = acc[c * NP + pix] + bs[m][c];
        acc[c * NP + pix] = 0.f;
        bs[m][c] = 0.f;
        neumaier(sum[m][c], comp[m][c], v);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < PX; ++m) {
    const int gx = x0 + pc, gy = y0 + pr0 + m;
    if (gx < tk.W && gy < tk.H) {
      float *o = img + 3 * ((size_t)gy * tk.W + gx);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float v = sum[m][c] + comp[m][c];
        if (multi)
          unsafeAtomicAdd(o + c, v);
        else
          o[c] += v;
      }
    }
  }
}

constexpr int kLargeTile = 64;
constexpr int kLargeThreads = 512;
constexpr int kLargePx = kLargeTile * kLargeTile / kLargeThreads;  // 8 rows per lane

__global__ __launch_bounds__(kLargeThreads) void k_splat_large(
    const Item *__restrict__ items, const uint32_t *__restrict__ pairs,
    const float4 *__restrict__ rec, const uint32_t *__restrict__ counts, int cchunk, TileK tk,
    float *__restrict__ img) {
  __shared__ float g_ox[kLargeThreads], g_fx[kLargeThreads], g_oy[kLargeThreads],
      g_fy[kLargeThreads], g_is2[kLargeThreads];
  __shared__ float g_a0[kLargeThreads], g_a1[kLargeThreads], g_a2[kLargeThreads];
  __shared__ uint32_t g_box[kLargeThreads];
  __shared__ int g_count;

  const Item it = items[blockIdx.x];
  const int cb = (int)it.x - tk.n_tiles;
  const int x0 = (cb % tk.nctx) * kLargeTile, y0 = (cb / tk.nctx) * kLargeTile;
  const bool multi = counts[it.x] > (uint32_t)cchunk;
  const int tid = threadIdx.x;
  const int pc = tid % kLargeTile;
  const int pr0 = (tid / kLargeTile) * kLargePx;  // a wave = one 64 x 8 strip
  const float nu2 = tk.nu * tk.nu;

  float sum[kLargePx][3], comp[kLargePx][3], bs[kLargePx][3];
#pragma unroll
  for (int m = 0; m < kLargePx; ++m)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sum[m][c] = 0.f;
      comp[m][c] = 0.f;
      bs[m][c] = 0.f;
    }

  for (uint32_t base = it.y; base < it.z; base += kLargeThreads) {
    if (tid == 0) g_count = 0;
    __syncthreads();
    const uint32_t k = base + tid;
    if (k < it.z) {
      const uint32_t pid = pairs[k];
      const float4 r0 = rec[2 * (size_t)pid];
      const float4 r1 = rec[2 * (size_t)pid + 1];
      int i0, i1, j0, j1;
      if (record_box(r0.x, r0.y, r0.z, r0.w, r1.x, tk.nu, tk.W, tk.H, i0, i1, j0, j1)) {
        const int li0 = max(i0 - x0, 0), li1 = min(i1 - x0, kLargeTile - 1);
        const int lj0 = max(j0 - y0, 0), lj1 = min(j1 - y0, kLargeTile - 1);
        if (li0 <= li1 && lj0 <= lj1) {
          const int slot = atomicAdd(&g_count, 1);
          g_ox[slot] = r0.x - (float)x0;
          g_fx[slot] = 0.5f - r0.y;
          g_oy[slot] = r0.z - (float)y0;
          g_fy[slot] = 0.5f - r0.w;
          g_is2[slot] = 1.0f / (r1.x * r1.x);
          g_a0[slot] = r1.y;
          g_a1[slot] = r1.z;
          g_a2[slot] = r1.w;
          g_box[slot] = pack_box(li0, li1, lj0, lj1);
        }
      }
    }
    __syncthreads();
    const int ng = g_count;
    for (int g = 0; g < ng; ++g) {
      const uint32_t bx = g_box[g];
      const int li0 = bx & 0xff, li1 = (bx >> 8) & 0xff, lj0 = (bx >> 16) & 0xff,
                lj1 = bx >> 24;
      if (lj1 < pr0 || lj0 > pr0 + kLargePx - 1) continue;  // uniform across the wave
      if (pc < li0 || pc > li1) continue;
      const float dx = ((float)pc - g_ox[g]) + g_fx[g];
      const float dx2 = dx * dx;
      const float is2 = g_is2[g], oy = g_oy[g], fy = g_fy[g];
      const float a0 = g_a0[g], a1 = g_a1[g], a2 = g_a2[g];
#pragma unroll
      for (int m = 0; m < kLargePx; ++m) {
        const int row = pr0 + m;
        if (row < lj0 || row > lj1) continue;
        const float dy = ((float)row - oy) + fy;
        const float q = (dx2 + dy * dy) * is2;
        if (q <= nu2) {
          const float e = __expf(-q);
          bs[m][0] += a0 * e;
          bs[m][1] += a1 * e;
          bs[m][2] += a2 * e;
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kLargePx; ++m)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        neumaier(sum[m][c], comp[m][c], bs[m][c]);
        bs[m][c] = 0.f;
      }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < kLargePx; ++m) {
    const int gx = x0 + pc, gy = y0 + pr0 + m;
    if (gx < tk.W && gy < tk.H) {
      float *o = img + 3 * ((size_t)gy * tk.W + gx);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float v = sum[m][c] + comp[m][c];
        if (multi)
          unsafeAtomicAdd(o + c, v);
        else
          o[c] += v;
      }
    }
  }
}

template <int T>
__global__ __launch_bounds__(kBlock) void k_composite(const Item *__restrict__ items,
                                                      const unsigned long long *__restrict__ keys,
                                                      const float4 *__restrict__ rec,
                                                      const float2 *__restrict__ rec2,
                                                      const uint32_t *__restrict__ counts,
                                                      int chunk, TileK tk,
                                                      float *__restrict__ img,
                                                      float4 *__restrict__ partial) {
  constexpr int NP = T * T;
  constexpr int PX = NP / kBlock;
  constexpr int WROWS = (64 / T) * PX;
  __shared__ float g_ox[kBlock], g_fx[kBlock], g_oy[kBlock], g_fy[kBlock], g_is2[kBlock];
  __shared__ float g_a0[kBlock], g_a1[kBlock], g_a2[kBlock], g_ap[kBlock];
  __shared__ uint32_t g_box[kBlock];

  const Item it = items[blockIdx.x];
  const int tx = (int)it.x % tk.ntx, ty = (int)it.x / tk.ntx;
  const int x0 = tx * T, y0 = ty * T;
  const bool multi = counts[it.x] > (uint32_t)chunk;
  const int tid = threadIdx.x;
  const int pc = tid % T;
  const int pr0 = (tid / T) * PX;
  const int wr0 = (tid / 64) * WROWS, wr1 = wr0 + WROWS - 1;
  const float nu2 = tk.nu * tk.nu;

  float C[PX][3], Cc[PX][3], Cb[PX][3], Tr[PX];
#pragma unroll
  for (int m = 0; m < PX; ++m) {
    Tr[m] = 1.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      C[m][c] = 0.f;
      Cc[m][c] = 0.f;
      Cb[m][c] = 0.f;
    }
  }
  for (uint32_t base = it.y; base < it.z; base += kBlock) {
    const uint32_t k = base + tid;
    uint32_t box = pack_box(1, 0, 1, 0);  // empty unless set below (li0 > li1)
    if (k < it.z) {
      const uint32_t pid = (uint32_t)(keys[k] & 0xffffffffull);
      const float4 r0 = rec[2 * (size_t)pid];
      const float4 r1 = rec[2 * (size_t)pid + 1];
      int i0, i1, j0, j1;
      if (record_box(r0.x, r0.y, r0.z, r0.w, r1.x, tk.nu, tk.W, tk.H, i0, i1, j0, j1)) {
        const int li0 = max(i0 - x0, 0), li1 = min(i1 - x0, T - 1);
        const int lj0 = max(j0 - y0, 0), lj1 = min(j1 - y0, T - 1);
        if (li0 <= li1 && lj0 <= lj1) {
          box = pack_box(li0, li1, lj0, lj1);
          g_ox[tid] = r0.x - (float)x0;
          g_fx[tid] = 0.5f - r0.y;
          g_oy[tid] = r0.z - (float)y0;
          g_fy[tid] = 0.5f - r0.w;
          g_is2[tid] = 1.0f / (r1.x * r1.x);
          g_a0[tid] = r1.y;
          g_a1[tid] = r1.z;
          g_a2[tid] = r1.w;
          g_ap[tid] = rec2[pid].x;
        }
      }
    }
    g_box[tid] = box;
    __syncthreads();
    const int nb = (int)min((uint32_t)kBlock, it.z - base);
    for (int g = 0; g < nb; ++g) {
      const uint32_t bx = g_box[g];
      const int li0 = bx & 0xff, li1 = (bx >> 8) & 0xff, lj0 = (bx >> 16) & 0xff,
                lj1 = bx >> 24;
      if (li0 > li1 || lj1 < wr0 || lj0 > wr1) continue;  // uniform across the wave
      if (pc < li0 || pc > li1) continue;
      const float dx = ((float)pc - g_ox[g]) + g_fx[g];
      const float dx2 = dx * dx;
      const float is2 = g_is2[g], oy = g_oy[g], fy = g_fy[g], ap = g_ap[g];
#pragma unroll
      for (int m = 0; m < PX; ++m) {
        const int row = pr0 + m;
        if (row < lj0 || row > lj1) continue;
        const float dy = ((float)row - oy) + fy;
        const float q = (dx2 + dy * dy) * is2;
        if (q <= nu2) {
          const float e = __expf(-q);
          const float x = ap * e;
          const float em = expm1f(-x);                       // exp(-x) - 1
          const float w = (x > 1e-6f) ? (-em / x) : (1.0f - 0.5f * x);  // (1 - e^-x) / x
          const float tw = Tr[m] * e * w;
          Cb[m][0] += tw * g_a0[g];
          Cb[m][1] += tw * g_a1[g];
          Cb[m][2] += tw * g_a2[g];
          Tr[m] *= (1.0f + em);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < PX; ++m)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        neumaier(C[m][c], Cc[m][c], Cb[m][c]);
        Cb[m][c] = 0.f;
      }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < PX; ++m) {
    const int lx = pc, ly = pr0 + m;
    if (multi) {
      partial[(size_t)blockIdx.x * NP + ly * T + lx] =
          make_float4(C[m][0] + Cc[m][0], C[m][1] + Cc[m][1], C[m][2] + Cc[m][2], Tr[m]);
    } else {
      const int gx = x0 + lx, gy = y0 + ly;
      if (gx < tk.W && gy < tk.H) {
        float *o = img + 3 * ((size_t)gy * tk.W + gx);
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = C[m][c] + Cc[m][c];
      }
    }
  }
}

// Ordered merge of the partial tiles of a long sorted list: chunk c sees the
// light of chunks 0..c-1 through their transmittance.
template <int T>
__global__ __launch_bounds__(kBlock) void k_composite_merge(const Item *__restrict__ items,
                                                            const uint32_t *__restrict__ counts,
                                                            int chunk, TileK tk,
                                                            const float4 *__restrict__ partial,
                                                            float *__restrict__ img) {
  constexpr int NP = T * T;
  const Item it = items[blockIdx.x];
  const uint32_t cnt = counts[it.x];
  if (it.w != 0 || cnt <= (uint32_t)chunk) return;
  const int nch = (int)((cnt + (uint32_t)chunk - 1) / (uint32_t)chunk);
  const int tx = (int)it.x % tk.ntx, ty = (int)it.x / tk.ntx;
  for (int p = threadIdx.x; p < NP; p += kBlock) {
    float c0 = 0.f, c1 = 0.f, c2 = 0.f, tr = 1.f;
    for (int c = 0; c < nch; ++c) {
      const float4 v = partial[(size_t)(blockIdx.x + c) * NP + p];
      c0 += tr * v.x;
      c1 += tr * v.y;
      c2 += tr * v.z;
      tr *= v.w;
    }
    const int gx = tx * T + p % T, gy = ty * T + p / T;
    if (gx < tk.W && gy < tk.H) {
      float *o = img + 3 * ((size_t)gy * tk.W + gx);
      o[0] = c0;
      o[1] = c1;
      o[2] = c2;
    }
  }
}

}  // namespace

hipError_t launch_splat_add(int tile, const Item *items, int n_items, const uint32_t *pairs,
                            const float *rec, const uint32_t *counts, int chunk,
                            const TileK &tk, int scat_max, float *img, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const float4 *r = reinterpret_cast<const float4 *>(rec);
  if (tile == 16)
    hipLaunchKernelGGL(k_splat_add<16>, dim3(n_items), dim3(kBlock), 0, s, items, pairs, r, counts,
                       chunk, tk, scat_max, img);
  else if (tile == 32)
    hipLaunchKernelGGL(k_splat_add<32>, dim3(n_items), dim3(kBlock), 0, s, items, pairs, r, counts,
                       chunk, tk, scat_max, img);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_splat_large(const Item *items, int n_items, const uint32_t *pairs,
                              const float *rec, const uint32_t *counts, int cchunk,
                              const TileK &tk, float *img, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  if (tk.ctile != kLargeTile) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_splat_large, dim3(n_items), dim3(kLargeThreads), 0, s, items, pairs,
                     reinterpret_cast<const float4 *>(rec), counts, cchunk, tk, img);
  return hipGetLastError();
}

hipError_t launch_composite(int tile, const Item *items, int n_items,
                            const unsigned long long *keys, const float *rec, const float *rec2,
                            const uint32_t *counts, int chunk, const TileK &tk, float *img,
                            float *partial, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const float4 *r = reinterpret_cast<const float4 *>(rec);
  const float2 *r2 = reinterpret_cast<const float2 *>(rec2);
  float4 *pp = reinterpret_cast<float4 *>(partial);
  if (tile == 16)
    hipLaunchKernelGGL(k_composite<16>, dim3(n_items), dim3(kBlock), 0, s, items, keys, r, r2,
                       counts, chunk, tk, img, pp);
  else if (tile == 32)
    hipLaunchKernelGGL(k_composite<32>, dim3(n_items), dim3(kBlock), 0, s, items, keys, r, r2,
                       counts, chunk, tk, img, pp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_composite_merge(int tile, const Item *items, int n_items,
                                  const uint32_t *counts, int chunk, const TileK &tk,
                                  const float *partial, float *img, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const float4 *pp = reinterpret_cast<const float4 *>(partial);
  if (tile == 16)
    hipLaunchKernelGGL(k_composite_merge<16>, dim3(n_items), dim3(kBlock), 0, s, items, counts,
                       chunk, tk, pp, img);
  else if (tile == 32)
    hipLaunchKernelGGL(k_composite_merge<32>, dim3(n_items), dim3(kBlock), 0, s, items, counts,
                       chunk, tk, pp, img);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace spl
