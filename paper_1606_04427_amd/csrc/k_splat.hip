// Render stage (Sect. 3.1: each tile's list is rendered by one worker that
// owns the tile's pixels; Sect. 3.2.2: drawing adds colour x contribution to
// the pixel).  One workgroup per work item = one chunk of one tile's list;
// the tile's pixels live in registers and LDS, so no two workgroups share a
// pixel except the chunks of one long list, which merge by hardware float
// atomics (additive) or by an ordered merge of partial (colour,
// transmittance) tiles (sorted).
//
// k_splat_add<T>   additive modes, T x T tile, 256 lanes.  Each batch of list
//                  entries is loaded once, one entry per lane, and each
//                  entry's box inside the tile is cut into 4 x 4 windows
//                  listed in LDS (offsets from a prefix sum, no atomics).
//                  16-lane groups take the windows round-robin, one pixel per
//                  lane, keep running sums while a group's consecutive
//                  windows coincide (dense cluster cores) and add them into a
//                  32-bit fixed-point LDS accumulator with integer atomics
//                  (LDS FP32 atomics are ~40x slower on this hardware).  After
//                  every batch the accumulator is folded into per-pixel
//                  Neumaier-compensated FP32 sums.
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

// One list entry's box inside a tile is cut into 4 x 4 windows.  A window
// work item is a 32-bit word: entry slot in the batch (8 bits), window origin
// in the tile (x, y: 6 bits each), valid width and height minus one (2 bits
// each).
//
// Accumulation is in 32-bit fixed point: per batch, the scale 2^S is chosen so
// that the batch's summed amplitude (sum over entries of the largest colour
// channel) stays below 2^30, so no pixel sum can overflow; one quantum is at
// most 2^-31 of that sum.  LDS integer atomics are cheap on this hardware,
// LDS FP32 atomics are not.  Integer sums are also independent of the order in
// which the groups add.
template <int T, int BATCH>
__device__ __forceinline__ void splat_add_item(const Item it, const uint32_t *__restrict__ pairs,
                                               const float4 *__restrict__ rec,
                                               const uint32_t *__restrict__ counts, int chunk,
                                               const TileK &tk, float *__restrict__ img) {
  constexpr int NP = T * T;
  constexpr int PX = NP / kBlock;            // pixels per lane in the fold
  constexpr int MAXWIN = (T / 4) * (T / 4);  // windows of a box that fills the tile
  constexpr int NLW = BATCH / 64;            // waves that load entries
  constexpr float kLog2e = 1.4426950408889634f;
  __shared__ int acc[3 * NP];
  __shared__ float4 s_geo[BATCH];  // x offset, y offset, log2(e)/sigma^2, box origin
  __shared__ float4 s_col[BATCH];  // premultiplied colour
  __shared__ uint32_t s_win[BATCH * MAXWIN];
  __shared__ int s_wsum[4];
  __shared__ float s_asum[4];

  const int tx = (int)it.x % tk.ntx, ty = (int)it.x / tk.ntx;
  const int x0 = tx * T, y0 = ty * T;
  const bool multi = counts[it.x] > (uint32_t)chunk;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int grp = tid >> 4, kx = tid & 3, ky = (tid >> 2) & 3;
  const float qmax = tk.nu * tk.nu * kLog2e;

  float sum[PX][3], comp[PX][3];
#pragma unroll
  for (int m = 0; m < PX; ++m)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sum[m][c] = 0.f;
      comp[m][c] = 0.f;
    }
  for (int i = tid; i < 3 * NP; i += kBlock) acc[i] = 0;

  for (uint32_t base = it.y; base < it.z; base += BATCH) {
    // phase 1: one list entry per loading lane -> box in the tile, constants
    const uint32_t k = base + tid;
    int nwin = 0, nwx = 1, ex_li0 = 0, ex_li1 = 0, ex_lj0 = 0, ex_lj1 = 0;
    float amax = 0.f;
    if (tid < BATCH && k < it.z) {
      const uint32_t pid = pairs[k];
      const float4 r0 = rec[2 * (size_t)pid];
      const float4 r1 = rec[2 * (size_t)pid + 1];
      int i0, i1, j0, j1;
      if (record_box(r0.x, r0.y, r0.z, r0.w, r1.x, tk.nu, tk.W, tk.H, i0, i1, j0, j1)) {
        const int li0 = max(i0 - x0, 0), li1 = min(i1 - x0, T - 1);
        const int lj0 = max(j0 - y0, 0), lj1 = min(j1 - y0, T - 1);
        if (li0 <= li1 && lj0 <= lj1) {
          // offset of pixel centre (li0 + u, lj0 + v) from the particle is
          // (cx + u, cy + v); the integer parts subtract exactly
          const float cx = ((float)(li0 + x0) - r0.x) + (0.5f - r0.y);
          const float cy = ((float)(lj0 + y0) - r0.z) + (0.5f - r0.w);
          s_geo[tid] = make_float4(cx, cy, kLog2e / (r1.x * r1.x),
                                   __uint_as_float((uint32_t)li0 | ((uint32_t)lj0 << 16)));
          s_col[tid] = make_float4(r1.y, r1.z, r1.w, 0.f);
          nwx = (li1 - li0) / 4 + 1;
          nwin = nwx * ((lj1 - lj0) / 4 + 1);
          ex_li1 = li1;
          ex_lj1 = lj1;
          ex_li0 = li0;
          ex_lj0 = lj0;
          amax = fmaxf(fmaxf(fabsf(r1.y), fabsf(r1.z)), fabsf(r1.w));
        }
      }
    }
    // window offsets: inclusive scan inside each wave, wave totals in LDS;
    // batch amplitude bound: sum of each entry's largest channel
    int incl = nwin;
    float asum = amax;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
      asum += __shfl_xor(asum, d);
    }
    if (wave < NLW && lane == 63) s_wsum[wave] = incl;
    if (wave < NLW && lane == 0) s_asum[wave] = asum;
    __syncthreads();
    int woff = 0, total = 0;
    float amp_sum = 0.f;
#pragma unroll
    for (int w = 0; w < NLW; ++w) {
      if (w < wave) woff += s_wsum[w];
      total += s_wsum[w];
      amp_sum += s_asum[w];
    }
    int ex = 0;
    (void)frexpf(amp_sum, &ex);  // amp_sum <= 2^ex
    const int S = 30 - ex;       // batch sums stay below 2^30
    for (int w = 0, o = woff + incl - nwin; w < nwin; ++w, ++o) {
      const int wx0 = ex_li0 + 4 * (w % nwx), wy0 = ex_lj0 + 4 * (w / nwx);
      const int ww = min(3, ex_li1 - wx0), wh = min(3, ex_lj1 - wy0);
      s_win[o] = (uint32_t)tid | ((uint32_t)wx0 << 8) | ((uint32_t)wy0 << 14) |
                 ((uint32_t)ww << 20) | ((uint32_t)wh << 22);
    }
    __syncthreads();

    // phase 2: 16-lane groups take windows round-robin, one pixel per lane,
    // and keep running sums while a group's consecutive windows coincide
    {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
      int cur = -1;  // the lane's pixel in the current window; NP = outside
      for (int e = grp; e < total; e += 16) {
        const uint32_t w = s_win[e];
        const int slot = (int)(w & 0xffu);
        const float4 g = s_geo[slot];
        const float4 col = s_col[slot];
        const int px = (int)((w >> 8) & 63u) + kx, py = (int)((w >> 14) & 63u) + ky;
        const int pix = (px < T && py < T) ? py * T + px : NP;
        if (pix != cur) {
          if (cur >= 0 && cur < NP) {
            atomicAdd(&acc[cur], (int)rintf(ldexpf(a0, S)));
            atomicAdd(&acc[NP + cur], (int)rintf(ldexpf(a1, S)));
            atomicAdd(&acc[2 * NP + cur], (int)rintf(ldexpf(a2, S)));
          }
          cur = pix;
          a0 = a1 = a2 = 0.f;
        }
        if (kx <= (int)((w >> 20) & 3u) && ky <= (int)((w >> 22) & 3u)) {
          const uint32_t org = __float_as_uint(g.w);
          const float dx = g.x + (float)(px - (int)(org & 0xffffu));
          const float dy = g.y + (float)(py - (int)(org >> 16));
          const float q = (dx * dx + dy * dy) * g.z;
          if (q <= qmax) {
            const float e2 = exp2f(-q);
            a0 += col.x * e2;
            a1 += col.y * e2;
            a2 += col.z * e2;
          }
        }
      }
      if (cur >= 0 && cur < NP) {
        atomicAdd(&acc[cur], (int)rintf(ldexpf(a0, S)));
        atomicAdd(&acc[NP + cur], (int)rintf(ldexpf(a1, S)));
        atomicAdd(&acc[2 * NP + cur], (int)rintf(ldexpf(a2, S)));
      }
    }
    __syncthreads();
    // phase 3: fold the batch sums into the compensated per-pixel sums
#pragma unroll
    for (int m = 0; m < PX; ++m) {
      const int pix = tid + m * kBlock;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int v = acc[c * NP + pix];
        acc[c * NP + pix] = 0;
        neumaier(sum[m][c], comp[m][c], ldexpf((float)v, -S));
      }
    }
  }
#pragma unroll
  for (int m = 0; m < PX; ++m) {
    const int pix = tid + m * kBlock;
    const int gx = x0 + pix % T, gy = y0 + pix / T;
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

template <int T, int BATCH>
__global__ __launch_bounds__(kBlock, 6) void k_splat_add(const Item *__restrict__ items,
                                                      const uint32_t *__restrict__ pairs,
                                                      const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ counts,
                                                      int chunk, TileK tk,
                                                      float *__restrict__ img) {
  splat_add_item<T, BATCH>(items[blockIdx.x], pairs, rec, counts, chunk, tk, img);
}

// Persistent form for many views: workgroups take (view, tile chunk) items
// from a device counter until the queue is empty; every workgroup exits.
template <int T, int BATCH>
__global__ __launch_bounds__(kBlock, 6) void k_splat_add_views(const ViewK *__restrict__ views,
                                                            const Item *__restrict__ items,
                                                            const uint32_t *__restrict__ n_items,
                                                            uint32_t *__restrict__ next,
                                                            int chunk) {
  __shared__ uint32_t s_idx;
  const uint32_t n = *n_items;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(next, 1u);
    __syncthreads();
    const uint32_t idx = s_idx;
    __syncthreads();
    if (idx >= n) break;
    Item it = items[idx];
    const ViewK &v = views[it.x >> 24];
    it.x &= 0xffffffu;
    splat_add_item<T, BATCH>(it, v.pairs, v.rec, v.counts, chunk, v.tk, v.img);
    __syncthreads();
  }
}

constexpr int kLargeTile = 64;
constexpr int kLargeThreads = 512;
constexpr int kLargePx = kLargeTile * kLargeTile / kLargeThreads;  // 8 rows per lane

__device__ __forceinline__ void splat_large_item(const Item it, const uint32_t *__restrict__ pairs,
                                                 const float4 *__restrict__ rec,
                                                 const uint32_t *__restrict__ counts, int cchunk,
                                                 const TileK &tk, float *__restrict__ img) {
  __shared__ float g_ox[kLargeThreads], g_fx[kLargeThreads], g_oy[kLargeThreads],
      g_fy[kLargeThreads], g_is2[kLargeThreads];
  __shared__ float g_a0[kLargeThreads], g_a1[kLargeThreads], g_a2[kLargeThreads];
  __shared__ uint32_t g_box[kLargeThreads];
  __shared__ int g_count;

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

__global__ __launch_bounds__(kLargeThreads) void k_splat_large(
    const Item *__restrict__ items, const uint32_t *__restrict__ pairs,
    const float4 *__restrict__ rec, const uint32_t *__restrict__ counts, int cchunk, TileK tk,
    float *__restrict__ img) {
  splat_large_item(items[blockIdx.x], pairs, rec, counts, cchunk, tk, img);
}

__global__ __launch_bounds__(kLargeThreads) void k_splat_large_views(
    const ViewK *__restrict__ views, const Item *__restrict__ items,
    const uint32_t *__restrict__ n_items, uint32_t *__restrict__ next, int cchunk) {
  __shared__ uint32_t s_idx;
  const uint32_t n = *n_items;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(next, 1u);
    __syncthreads();
    const uint32_t idx = s_idx;
    __syncthreads();
    if (idx >= n) break;
    Item it = items[idx];
    const ViewK &v = views[it.x >> 24];
    it.x &= 0xffffffu;
    splat_large_item(it, v.pairs, v.rec, v.counts, cchunk, v.tk, v.img);
    __syncthreads();
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
                            const TileK &tk, float *img, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const float4 *r = reinterpret_cast<const float4 *>(rec);
  if (tile == 16)
    hipLaunchKernelGGL((k_splat_add<16, 256>), dim3(n_items), dim3(kBlock), 0, s, items, pairs, r,
                       counts, chunk, tk, img);
  else if (tile == 32)
    hipLaunchKernelGGL((k_splat_add<32, 128>), dim3(n_items), dim3(kBlock), 0, s, items, pairs, r,
                       counts, chunk, tk, img);
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

hipError_t launch_splat_views(int tile, const ViewK *views, const Item *fine, const uint32_t *n_fine,
                              uint32_t *next_fine, const Item *large, const uint32_t *n_large,
                              uint32_t *next_large, int chunk, int cchunk, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_splat_large_views, dim3(grid), dim3(kLargeThreads), 0, s, views, large,
                     n_large, next_large, cchunk);
  if (tile == 16)
    hipLaunchKernelGGL((k_splat_add_views<16, 256>), dim3(grid), dim3(kBlock), 0, s, views, fine,
                       n_fine, next_fine, chunk);
  else if (tile == 32)
    hipLaunchKernelGGL((k_splat_add_views<32, 128>), dim3(grid), dim3(kBlock), 0, s, views, fine,
                       n_fine, next_fine, chunk);
  else
    return hipErrorInvalidValue;
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
