// Render stage (Sect. 3.1: each tile's list is rendered by one worker that
// owns the tile's pixels; Sect. 3.2.2: drawing adds colour x contribution to
// the pixel).  One workgroup per work item = one chunk of one tile's list;
// the tile's pixels live in registers and LDS, so no two workgroups share a
// pixel except the chunks of one long list, which merge by hardware float
// atomics (additive) or by an ordered merge of partial (colour,
// transmittance) tiles (sorted, and the additive sum in list order).
//
// k_splat_add<T>   additive modes, T x T tile, 256 lanes.  Each batch of list
//                  entries is staged in LDS and appended to the lists of the
//                  4 x 4 micro-tiles it meets; the lists, laid end to end, are
//                  cut into 32 near-equal ranges for the 8-lane groups (two
//                  pixels per lane), with running sums in registers flushed into a
//                  32-bit fixed-point LDS accumulator at micro-tile changes.
//                  Batch sums fold into per-pixel FP64 sums in registers.
// k_splat_large    the large-particle path: 64 x 64 px tiles, 512 lanes, 8
//                  pixels per lane, gather only (a large particle covers most
//                  of the pixels it is tested against).
// k_composite<T,A> sorted mode (A) and the additive sum in list order (not
//                  A: no absorption): staging as above, in-order micro-tile
//                  lists built by ballots, walked in near-equal ranges by
//                  8-lane groups (two pixels per lane); front-to-back slab
//                  compositing of each list piece, pieces merged per pixel in
//                  list order.
#include <type_traits>

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

// Nearest integer, halves rounded up (one instruction: floor(x + 0.5)).
__device__ __forceinline__ int round_half_up(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ uint32_t pack_box(int a0, int a1, int b0, int b1) {
  return (uint32_t)a0 | ((uint32_t)a1 << 8) | ((uint32_t)b0 << 16) | ((uint32_t)b1 << 24);
}

// The 4 x 4 px micro-tiles of a tile (MX per row) whose rectangle of pixel
// centres the truncation disc of radius R can reach, one bit each (bit
// qy * MX + qx), with a margin over the rounding of this test and of the
// evaluation.  ux, uy: the particle centre minus half a pixel, in pixels
// from the tile origin.  Lengths below are in micro-tiles (4 px): the centre
// (cx, cy) and the radius with margin rq; row band qy (pixel rows 4 qy ..
// 4 qy + 3) lies at ey = max(qy - cy, cy - qy - 3/4, 0) from the centre and
// is reached when ey <= rq, and then so are its columns a..b, those within
// sqrt(rq^2 - ey^2) the same way: one square root per row band instead of a
// test per micro-tile.
template <int MX, typename MT>
__device__ __forceinline__ MT disc_micro_tiles(float ux, float uy, float R) {
  const float cx = ux * 0.25f, cy = uy * 0.25f;
  const float r2q = fmaf(R * R, 1.0001f, 1e-3f) * 0.0625f;
  const float rq = __builtin_amdgcn_sqrtf(r2q);
  const int qy0 = max((int)ceilf((cy - 0.75f) - rq), 0);
  const int qy1 = min((int)floorf(cy + rq), MX - 1);
  const float ca = cx - 0.75f;
  MT mask = 0;
  float fy = (float)qy0 - cy;
  for (int qy = qy0; qy <= qy1; ++qy, fy += 1.f) {
    const float ey = fmaxf(fmaxf(fy, -0.75f - fy), 0.f);
    const float hw = __builtin_amdgcn_sqrtf(fmaxf(fmaf(-ey, ey, r2q), 0.f));
    const int a = max((int)ceilf(ca - hw), 0);
    const int b = min((int)floorf(cx + hw), MX - 1);
    if (a <= b) mask |= (MT)(((MT)1 << (b - a + 1)) - 1) << (a + qy * MX);
  }
  return mask;
}

// A batch of up to 256 list entries is staged in LDS (offsets, width,
// premultiplied colour).  The tile is split into 4 x 4 micro-tiles and each
// staged entry appends itself to the list of every micro-tile its truncation
// disc can reach (LDS integer atomics; order inside a list is free for a
// sum).  Those micro-tiles are found row by row: the disc's half-width at the
// row band of micro-tiles gives the interval of micro-tile columns, so one
// square root per row band replaces a test per micro-tile, and the appends
// run over the set bits of the resulting mask.  The lists, laid end to end,
// are cut into 32 ranges whose lengths differ by at most one, one per 8-lane
// group; all groups step through their ranges together, one list entry per
// step, so the eight groups of a wave, which run in lockstep, take the same
// number of steps however unevenly the entries fall on the micro-tiles.  The
// per-step work is one compare for the end of the current list, the entry's
// staging offset and the Gaussian; the step that only the longer ranges take
// is peeled off the loop.  Two pixels per lane, rows r and r + 2 of one
// micro-tile column: the entry read from LDS and the horizontal distance
// serve both (LDS reads, not the vector ALU alone, bound the walk).  The
// running sums stay in registers while consecutive entries belong to the same
// micro-tile and are added into a 32-bit fixed-point LDS accumulator (integer
// atomics: neighbouring ranges may share a micro-tile) when the group moves
// on to the next non-empty list.  The staged colours carry the batch scale
// 2^S, which keeps the batch's summed peak amplitude below 2^30, so a flush
// only rounds and no pixel sum overflows.  After each batch the integer sums
// are folded into per-pixel FP64 sums in registers.
template <int T>
__device__ __forceinline__ void splat_add_item(const Item it, const uint32_t *__restrict__ pairs,
                                               const float4 *__restrict__ rec,
                                               const uint32_t *__restrict__ counts, int chunk,
                                               const TileK &tk, float *__restrict__ img) {
  constexpr int NP = T * T;
  constexpr int PX = NP / kBlock;      // pixels per lane in the fold
  constexpr int MX = T / 4;            // micro-tiles per tile row
  constexpr int NQ = MX * MX;          // micro-tiles per tile (16 or 64)
  constexpr float kLog2e = 1.4426950408889634f;
  constexpr float kRootLog2e = 1.2011224087864498f;  // sqrt(log2 e)
  constexpr float kHalfSpan = 0.5f * (float)(T - 1);  // tile centre, in pixels
  // micro-tile masks: bit qy * MX + qx
  using MT = typename std::conditional<(NQ > 32), uint64_t, uint32_t>::type;
  // with g = sqrt(log2 e)/sigma and pixel positions taken from the tile
  // centre (c = column - (T - 1)/2): the scaled offset g (x - X) of a pixel
  // centre from the particle is g c + ox, and the same down the column
  __shared__ float4 s_pos[kBlock];     // ox, oy, g, red x 2^S
  __shared__ float4 s_col[kBlock];     // green, blue x 2^S (first two words)
  // list entries: byte offsets into s_pos / s_col (16-bit, 16 px tiles) or
  // staging slots (8-bit, 32 px tiles, where the lists take 4x the LDS)
  using LT = typename std::conditional<T == 16, uint16_t, uint8_t>::type;
  constexpr int kShift = T == 16 ? 0 : 4;
  __shared__ __align__(4) LT s_list[NQ][kBlock];
  __shared__ int s_len[2][NQ];         // list lengths; batches alternate buffers
  __shared__ int s_start[NQ + 1];      // list offsets laid end to end
  // per list, the next non-empty list: its byte offset in s_list, length,
  // byte offset of its first pixel in s_iacc, own offset in this table; then
  // its first pixel's centred column and row (floats)
  __shared__ int4 s_nx[2 * NQ];
  __shared__ int s_iacc[3][NP];        // batch sums, fixed point
  __shared__ float s_amp[4];           // per-wave summed peak amplitudes

  const int tx = (int)it.x % tk.ntx, ty = (int)it.x / tk.ntx;
  const int x0 = tx * T, y0 = ty * T;
  const bool multi = counts[it.x] > (uint32_t)chunk;
  // walk: 8-lane groups; lane (lx, ly) of a group takes the micro-tile
  // pixels (lx, ly) and (lx, ly + 2)
  const int tid = threadIdx.x, grp = tid >> 3, l = tid & 7, wave = tid >> 6;
  const int lx = l & 3, ly = l >> 2;
  const float qmax = tk.nu * tk.nu * kLog2e;

  double acc[PX][3];
#pragma unroll
  for (int m = 0; m < PX; ++m)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[m][c] = 0.0;
  for (int i = tid; i < 3 * NP; i += kBlock) (&s_iacc[0][0])[i] = 0;
  if (tid < 2 * NQ) (&s_len[0][0])[tid] = 0;
  __syncthreads();

  int cur = 0;
  for (uint32_t base = it.y; base < it.z; base += kBlock, cur ^= 1) {
    int *const len = s_len[cur];
    // stage one list entry per lane, append it to the list of every
    // micro-tile its disc reaches, sum the peak amplitudes.  Listed records
    // are finite with sigma > 0 (the binning lists no other).
    const uint32_t k = base + tid;
    float amax = 0.f;
    float4 r1 = make_float4(0.f, 0.f, 0.f, 0.f);
    float g = 0.f, ox = 0.f, oy = 0.f;
    if (k < it.z) {
      const uint32_t pid = pairs[k];
      const float4 r0 = rec[2 * (size_t)pid];
      r1 = rec[2 * (size_t)pid + 1];
      g = kRootLog2e * __builtin_amdgcn_rcpf(r1.x);
      // the integer differences are exact; two roundings each
      ox = fmaf(kHalfSpan - (r0.x - (float)x0), g, (0.5f - r0.y) * g);
      oy = fmaf(kHalfSpan - (r0.z - (float)y0), g, (0.5f - r0.w) * g);
      amax = fmaxf(fmaxf(fabsf(r1.y), fabsf(r1.z)), fabsf(r1.w));
      MT mask = disc_micro_tiles<MX, MT>((r0.x - (float)x0) + (r0.y - 0.5f),
                                         (r0.z - (float)y0) + (r0.w - 0.5f), tk.nu * r1.x);
      while (mask) {
        const int q = NQ > 32 ? (int)__builtin_ctzll((unsigned long long)mask)
                              : (int)__builtin_ctz((unsigned)mask);
        mask &= mask - 1;
        s_list[q][atomicAdd(&len[q], 1)] = (LT)(tid << (4 - kShift));
      }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) amax += __shfl_xor(amax, o);
    if ((tid & 63) == 0) s_amp[wave] = amax;
    __syncthreads();
    int ex = 0;
    (void)frexpf(s_amp[0] + s_amp[1] + s_amp[2] + s_amp[3], &ex);  // sum <= 2^ex
    const int S = 30 - ex;
    // colours scaled by 2^S (exact); only the walk, after the next barrier,
    // reads them
    if (k < it.z) {
      s_pos[tid] = make_float4(ox, oy, g, ldexpf(r1.y, S));
      *reinterpret_cast<float2 *>(&s_col[tid]) = make_float2(ldexpf(r1.z, S), ldexpf(r1.w, S));
    }
    // list offsets and the next non-empty list of each list (one wave: NQ <= 64)
    if (tid < 64) {
      const int v = tid < NQ ? len[tid] : 0;
      int incl = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (tid >= o) incl += u;
      }
      const unsigned long long full = __ballot(v > 0);
      const unsigned long long later = tid < 63 ? full & (~0ull << (tid + 1)) : 0ull;
      // (a list with no later non-empty list is never left mid-walk)
      const int nq = later ? (int)__builtin_ctzll(later) : 0;
      const int nv = __shfl(v, nq);
      if (tid < NQ) {
        s_start[tid] = incl - v;
        const int nqx = nq % MX, nqy = nq / MX;
        s_nx[2 * tid] = make_int4(nq * kBlock * (int)sizeof(LT), nv,
                                  4 * (nqy * 4 * T + nqx * 4), nq * 32);
        s_nx[2 * tid + 1] = make_int4(__float_as_int((float)(nqx * 4) - kHalfSpan),
                                      __float_as_int((float)(nqy * 4) - kHalfSpan), 0, 0);
      }
      if (tid == NQ - 1) s_start[NQ] = incl;
    }
    __syncthreads();
    {
      // the lists laid end to end are cut into 32 ranges whose lengths differ
      // by at most one: every group takes `steps` entries, the first `rem`
      // groups one more
      const int total = s_start[NQ];
      const int steps = total >> 5, rem = total & 31;
      const int r0 = grp * steps + min(grp, rem);
      // the group's micro-tile at r0: the last list starting at or before it
      int q = 0;
#pragma unroll
      for (int h = NQ / 2; h >= 1; h >>= 1)
        if (s_start[q + h] <= r0) q += h;
      // lp: index in s_list of the next entry; le: end of the current list
      int lp = q * kBlock + (r0 - s_start[q]);
      int le = q * kBlock + (s_start[q + 1] - s_start[q]);
      // pb: byte offset of the lane's first pixel in each plane of s_iacc
      const int loff = 4 * (ly * T + lx);
      int pb = 4 * ((q / MX) * 4 * T + (q % MX) * 4) + loff;
      int qo = q * 32;  // byte offset of the list's entry in s_nx
      float px = (float)((q % MX) * 4 + lx) - kHalfSpan;
      float py = (float)((q / MX) * 4 + ly) - kHalfSpan;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f;
      // steps in blocks of four read the list at entry b + u (u = 0..3,
      // an immediate offset from the byte offset bo of entry b); the end
      // of the current list is at b + d
      constexpr int kLB = (int)sizeof(LT);
      const char *const s_lb = reinterpret_cast<const char *>(&s_list[0][0]);
      int bo = lp * kLB, d = le - lp;
      // the running sums into the fixed-point accumulator, rows r and r + 2
      auto flush = [&](const int b) {
        char *const acc_b = reinterpret_cast<char *>(&s_iacc[0][0]) + b;
        atomicAdd(reinterpret_cast<int *>(acc_b), round_half_up(a0));
        atomicAdd(reinterpret_cast<int *>(acc_b + 4 * NP), round_half_up(a1));
        atomicAdd(reinterpret_cast<int *>(acc_b + 8 * NP), round_half_up(a2));
        atomicAdd(reinterpret_cast<int *>(acc_b + 8 * T), round_half_up(b0));
        atomicAdd(reinterpret_cast<int *>(acc_b + 4 * NP + 8 * T), round_half_up(b1));
        atomicAdd(reinterpret_cast<int *>(acc_b + 8 * NP + 8 * T), round_half_up(b2));
      };
      auto step = [&](const int u) {
        if (d == u) {
          // next micro-tile: flush the running sums (already scaled by 2^S)
          flush(pb);
          a0 = a1 = a2 = 0.f;
          b0 = b1 = b2 = 0.f;
          const char *const nb = reinterpret_cast<const char *>(s_nx) + qo;
          const int4 n = *reinterpret_cast<const int4 *>(nb);
          const int4 nf = *reinterpret_cast<const int4 *>(nb + 16);
          qo = n.w;
          bo = n.x - u * kLB;
          d = u + n.y;
          pb = n.z + loff;
          px = __int_as_float(nf.x) + (float)lx;
          py = __int_as_float(nf.y) + (float)ly;
        }
        // byte offset of the entry's staging slot
        const int jb = (int)*reinterpret_cast<const LT *>(s_lb + bo + u * kLB) << kShift;
        const float4 p = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_pos) + jb);
        const float2 c = *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(s_col) + jb);
        // distances in units of sigma / sqrt(log2 e); two rows down adds 2 g
        const float dx = fmaf(px, p.z, p.x);
        const float dy = fmaf(py, p.z, p.y);
        const float dz = fmaf(2.f, p.z, dy);
        const float dx2 = dx * dx;
        const float qq = fmaf(dy, dy, dx2);
        const float qz = fmaf(dz, dz, dx2);
        // qq <= qmax keeps the result far above the denormal range, so
        // the hardware exponential needs no range fix-up
        const float e = (qq <= qmax) ? __builtin_amdgcn_exp2f(-qq) : 0.f;
        const float f = (qz <= qmax) ? __builtin_amdgcn_exp2f(-qz) : 0.f;
        a0 += p.w * e;
        a1 += c.x * e;
        a2 += c.y * e;
        b0 += p.w * f;
        b1 += c.x * f;
        b2 += c.y * f;
      };
      int t = 0;
      for (; t + 4 <= steps; t += 4) {  // uniform across the workgroup
        step(0);
        step(1);
        step(2);
        step(3);
        bo += 4 * kLB;
        d -= 4;
      }
      for (; t < steps; ++t) {
        step(0);
        bo += kLB;
        d -= 1;
      }
      if (grp < rem) step(0);
      if (steps > 0 || grp < rem) flush(pb);
    }
    // the other length buffer was last read before the previous batch's
    // final barrier and is next written after this batch's
    if (tid < NQ) s_len[cur ^ 1][tid] = 0;
    __syncthreads();
    // fold the batch sums into the per-pixel FP64 sums
#pragma unroll
    for (int m = 0; m < PX; ++m) {
      const int p2 = tid + m * kBlock;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int v = s_iacc[c][p2];
        s_iacc[c][p2] = 0;
        acc[m][c] += ldexp((double)v, -S);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < PX; ++m) {
    const int p2 = tid + m * kBlock;
    const int gx = x0 + p2 % T, gy = y0 + p2 / T;
    if (gx < tk.W && gy < tk.H) {
      float *o = img + 3 * ((size_t)gy * tk.W + gx);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float v = (float)acc[m][c];
        if (multi)
          unsafeAtomicAdd(o + c, v);
        else
          o[c] += v;
      }
    }
  }
}

// Eight workgroups per CU with 16 px tiles; the 32 px tiles' micro-tile
// lists take four times the LDS, which holds them to four.
template <int T>
__global__ __launch_bounds__(kBlock, T == 16 ? 8 : 4) void k_splat_add(const Item *__restrict__ items,
                                                      const uint32_t *__restrict__ pairs,
                                                      const float4 *__restrict__ rec,
                                                      const uint32_t *__restrict__ counts,
                                                      int chunk, TileK tk,
                                                      float *__restrict__ img) {
  splat_add_item<T>(items[blockIdx.x], pairs, rec, counts, chunk, tk, img);
}

// Persistent form for many views: workgroups take (view, tile chunk) items
// from a device counter until the queue is empty; every workgroup exits.
template <int T>
__global__ __launch_bounds__(kBlock, T == 16 ? 8 : 4) void k_splat_add_views(const ViewK *__restrict__ views,
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
    splat_add_item<T>(it, v.pairs, v.rec, v.counts, chunk, v.tk, v.img);
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

// Sorted mode.  Staging as in splat_add_item; each micro-tile's list is built
// by ballots in the depth order of the tile list.  The lists, laid end to
// end, are cut into 32 ranges whose lengths differ by at most one, one per
// 8-lane group (two pixels per lane, rows r and r + 2 of a micro-tile
// column, sharing the entry's LDS reads and horizontal distance), and walked
// in lockstep as in the additive kernel.  A group
// composites each piece of a micro-tile list it meets front to back from
// (C, T) = (0, 1): C += T E tau phi(a tau), T *= exp(-a tau), with
// phi(x) = (1 - e^-x)/x from a polynomial below x = 1/2 (no cancellation)
// and from the exponential above, and leaves the piece's
// (C, T) in LDS.  After the walk each lane merges, for its pixels, the pieces
// of the batch in list order into the running (C, T): C += T C_piece,
// T *= T_piece.  The pieces of one batch fill at most NQ + 31 slots: the
// (group, micro-tile) pairs of the walk form a staircase, so group + micro-tile
// numbers them.
// (KT: 64-bit (depth, index) keys with absorption, 32-bit indices without)
template <int T, bool kAbs, typename KT = typename std::conditional<kAbs, unsigned long long,
                                                                    uint32_t>::type>
__global__ __launch_bounds__(kBlock) void k_composite(const Item *__restrict__ items,
                                                      const KT *__restrict__ keys,
                                                      const KT *__restrict__ keys_b,
                                                      uint32_t sort_chunk,
                                                      const float4 *__restrict__ rec,
                                                      const float2 *__restrict__ rec2,
                                                      const uint32_t *__restrict__ counts,
                                                      int chunk, TileK tk,
                                                      float *__restrict__ img,
                                                      float4 *__restrict__ partial) {
  constexpr int NP = T * T;
  constexpr int PX = NP / kBlock;      // pixels per lane in the merge
  constexpr int MX = T / 4;
  constexpr int NQ = MX * MX;
  constexpr int MT = NQ / 16;          // lists built per 16-lane group
  constexpr int NS = NQ + 31;          // piece slots
  constexpr float kLog2e = 1.4426950408889634f;
  constexpr float kRootLog2e = 1.2011224087864498f;  // sqrt(log2 e)
  constexpr float kHalfSpan = 0.5f * (float)(T - 1);  // tile centre, in pixels
  // as in the additive splat: with g = sqrt(log2 e)/sigma and pixel positions
  // taken from the tile centre, the scaled offset of a pixel centre from the
  // particle is g c + ox (one FMA)
  __shared__ float4 s_pos[kBlock];     // ox, oy, g, -
  __shared__ float4 s_col[kBlock];     // -, colour
  __shared__ float s_ap[kBlock];       // a / (pi sigma^2)
  // micro-tiles each staged entry's truncation disc can reach, one bit each
  using MaskT = typename std::conditional<(NQ > 32), unsigned long long, uint32_t>::type;
  __shared__ MaskT s_mask[kBlock];
  __shared__ __align__(4) uint8_t s_list[NQ][kBlock];
  __shared__ int s_len[NQ];
  __shared__ int s_start[NQ + 1];
  __shared__ float4 s_piece[NS][16];   // per slot and micro-tile pixel: C rgb, T

  const Item it = items[blockIdx.x];
  const int tx = (int)it.x % tk.ntx, ty = (int)it.x / tk.ntx;
  const int x0 = tx * T, y0 = ty * T;
  const uint32_t cnt_tile = counts[it.x];
  const bool multi = cnt_tile > (uint32_t)chunk;
  // the buffer the list's merge passes left it in
  const KT *const src = (merge_passes(cnt_tile, sort_chunk) & 1) ? keys_b : keys;
  // list building: 16-lane groups; walk: 8-lane groups, lane (lx, ly) of a
  // group takes the micro-tile pixels (lx, ly) and (lx, ly + 2)
  const int tid = threadIdx.x, grp = tid >> 4, l = tid & 15, gw = grp & 3;
  const int wg = tid >> 3, wl = tid & 7, lx = wl & 3, ly = wl >> 2;
  const float qmax = tk.nu * tk.nu * kLog2e;

  // running (C, T) of the lane's pixels p2 = tid + m * kBlock
  float C[PX][3], Cc[PX][3], Tr[PX];
#pragma unroll
  for (int m = 0; m < PX; ++m) {
    Tr[m] = 1.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      C[m][c] = 0.f;
      Cc[m][c] = 0.f;
    }
  }
  for (uint32_t base = it.y; base < it.z; base += kBlock) {
    const uint32_t k = base + tid;
    MaskT mask = 0;
    if (k < it.z) {
      const uint32_t pid = (uint32_t)(src[k] & (KT)0xffffffffu);
      const float4 r0 = rec[2 * (size_t)pid];
      const float4 r1 = rec[2 * (size_t)pid + 1];
      // (listed records are finite with sigma > 0)
      const float g = kRootLog2e * __builtin_amdgcn_rcpf(r1.x);
      s_pos[tid] = make_float4(fmaf(kHalfSpan - (r0.x - (float)x0), g, (0.5f - r0.y) * g),
                               fmaf(kHalfSpan - (r0.z - (float)y0), g, (0.5f - r0.w) * g), g,
                               0.f);
      s_col[tid] = make_float4(0.f, r1.y, r1.z, r1.w);
      if (kAbs) s_ap[tid] = rec2[pid].x;
      // micro-tiles the disc can reach (the additive splat's test)
      mask = disc_micro_tiles<MX, MaskT>((r0.x - (float)x0) + (r0.y - 0.5f),
                                         (r0.z - (float)y0) + (r0.w - 0.5f), tk.nu * r1.x);
    }
    s_mask[tid] = mask;
    __syncthreads();
    // in-order list of every micro-tile, built by ballots of its group
    const int nb = (int)min((uint32_t)kBlock, it.z - base);
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int q = grp + 16 * m;
      int cnt = 0;
      for (int s0 = 0; s0 < nb; s0 += 16) {
        const int j = s0 + l;
        const bool hit = (s_mask[j] >> q) & 1;
        const uint32_t bits = (uint32_t)(__ballot(hit) >> (16 * gw)) & 0xffffu;
        if (hit) s_list[q][cnt + __popc(bits & ((1u << l) - 1u))] = (uint8_t)j;
        cnt += __popc(bits);
      }
      if (l == 0) s_len[q] = cnt;
    }
    __syncthreads();
    // list offsets (one wave: NQ <= 64)
    if (tid < 64) {
      const int v = tid < NQ ? s_len[tid] : 0;
      int incl = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (tid >= o) incl += u;
      }
      if (tid < NQ) s_start[tid] = incl - v;
      if (tid == NQ - 1) s_start[NQ] = incl;
    }
    __syncthreads();
    const int total = s_start[NQ];
    const int steps = total >> 5, rem = total & 31;
    {
      const int r0 = wg * steps + min(wg, rem);
      int q = 0;
#pragma unroll
      for (int h = NQ / 2; h >= 1; h >>= 1)
        if (s_start[q + h] <= r0) q += h;
      int lp = q * kBlock + (r0 - s_start[q]);
      int le = q * kBlock + (s_start[q + 1] - s_start[q]);
      float px = (float)((q % MX) * 4 + lx) - kHalfSpan;
      float py = (float)((q / MX) * 4 + ly) - kHalfSpan;
      // (C, T) of the piece for rows ly (a) and ly + 2 (b)
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, ta = 1.f;
      float b0 = 0.f, b1 = 0.f, b2 = 0.f, tb = 1.f;
      // one entry's slab, front to back, onto a pixel's running piece
      auto slab = [&](const float qq, const float ap, const float4 &c, float &c0, float &c1,
                      float &c2, float &tr) {
        if (!kAbs) {
          // no absorption (the ordered additive sum): T stays 1
          if (qq <= qmax) {
            const float e = __builtin_amdgcn_exp2f(-qq);
            c0 = fmaf(e, c.y, c0);
            c1 = fmaf(e, c.z, c1);
            c2 = fmaf(e, c.w, c2);
          }
          return;
        }
        if (qq <= qmax) {
          const float e = __builtin_amdgcn_exp2f(-qq);
          const float x = ap * e;
          float phi, em;  // phi(x), exp(-x) - 1
          if (x < 0.5f) {
            // degree-5 fit to phi on [0, 1/2], least squares in relative
            // error over Chebyshev nodes: 1.4e-9 relative in exact
            // arithmetic, 7e-8 in FP32 (as the degree-7 Taylor series)
            phi = fmaf(x, -1.121324371e-03f, 8.186993189e-03f);
            phi = fmaf(x, phi, -4.162891582e-02f);
            phi = fmaf(x, phi, 1.666622162e-01f);
            phi = fmaf(x, phi, -4.999997914e-01f);
            phi = fmaf(x, phi, 1.f);
            em = -x * phi;
          } else {
            em = __builtin_amdgcn_exp2f(-x * kLog2e) - 1.f;
            phi = -em * __builtin_amdgcn_rcpf(x);
          }
          const float tw = tr * e * phi;
          c0 = fmaf(tw, c.y, c0);
          c1 = fmaf(tw, c.z, c1);
          c2 = fmaf(tw, c.w, c2);
          tr = fmaf(tr, em, tr);
        }
      };
      auto put_piece = [&]() {
        s_piece[wg + q][ly * 4 + lx] = make_float4(a0, a1, a2, ta);
        s_piece[wg + q][(ly + 2) * 4 + lx] = make_float4(b0, b1, b2, tb);
      };
      auto step = [&]() {
        if (lp == le) {
          // end of this piece of the micro-tile's list
          put_piece();
          a0 = a1 = a2 = 0.f;
          b0 = b1 = b2 = 0.f;
          ta = tb = 1.f;
          do {
            ++q;
          } while (s_start[q + 1] == s_start[q]);
          lp = q * kBlock;
          le = lp + (s_start[q + 1] - s_start[q]);
          px = (float)((q % MX) * 4 + lx) - kHalfSpan;
          py = (float)((q / MX) * 4 + ly) - kHalfSpan;
        }
        const int j = (&s_list[0][0])[lp++];
        const float4 p = s_pos[j];
        const float4 c = s_col[j];
        const float ap = kAbs ? s_ap[j] : 0.f;
        // squared distances in units of sigma^2 / log2 e; two rows down
        // adds 2 g
        const float dx = fmaf(px, p.z, p.x);
        const float dy = fmaf(py, p.z, p.y);
        const float dz = fmaf(2.f, p.z, dy);
        const float dx2 = dx * dx;
        slab(fmaf(dy, dy, dx2), ap, c, a0, a1, a2, ta);
        slab(fmaf(dz, dz, dx2), ap, c, b0, b1, b2, tb);
      };
      for (int t = 0; t < steps; ++t) step();  // uniform across the workgroup
      if (wg < rem) step();
      if (steps > 0 || wg < rem) put_piece();
    }
    __syncthreads();
    // merge the pieces of each pixel's micro-tile in list order
    if (total > 0) {
      const int big = rem * (steps + 1);  // positions held by the longer ranges
      auto group_of = [&](int r) { return r < big ? r / (steps + 1) : rem + (r - big) / steps; };
#pragma unroll
      for (int m = 0; m < PX; ++m) {
        const int p2 = tid + m * kBlock;
        const int lpx = p2 % T, lpy = p2 / T;
        const int q = (lpy >> 2) * MX + (lpx >> 2), ql = (lpy & 3) * 4 + (lpx & 3);
        const int a = s_start[q], e = s_start[q + 1];
        if (a < e) {
          const int g1 = group_of(e - 1);
          for (int g = group_of(a); g <= g1; ++g) {
            const float4 pc = s_piece[g + q][ql];
            neumaier(C[m][0], Cc[m][0], Tr[m] * pc.x);
            neumaier(C[m][1], Cc[m][1], Tr[m] * pc.y);
            neumaier(C[m][2], Cc[m][2], Tr[m] * pc.z);
            Tr[m] *= pc.w;
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < PX; ++m) {
    const int p2 = tid + m * kBlock;
    const int lpx = p2 % T, lpy = p2 / T;
    if (multi) {
      partial[(size_t)blockIdx.x * NP + p2] =
          make_float4(C[m][0] + Cc[m][0], C[m][1] + Cc[m][1], C[m][2] + Cc[m][2], Tr[m]);
    } else {
      const int gx = x0 + lpx, gy = y0 + lpy;
      if (gx < tk.W && gy < tk.H) {
        float *o = img + 3 * ((size_t)gy * tk.W + gx);
        // (the additive sum adds into the image: a frame may come in chunks)
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = kAbs ? C[m][c] + Cc[m][c] : o[c] + (C[m][c] + Cc[m][c]);
      }
    }
  }
}

// Ordered merge of the partial tiles of a long sorted list: chunk c sees the
// light of chunks 0..c-1 through their transmittance (all 1 in the ordered
// additive sum, which adds the result into the image).
template <int T, bool kAbs>
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
      o[0] = kAbs ? c0 : o[0] + c0;
      o[1] = kAbs ? c1 : o[1] + c1;
      o[2] = kAbs ? c2 : o[2] + c2;
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
    hipLaunchKernelGGL((k_splat_add<16>), dim3(n_items), dim3(kBlock), 0, s, items, pairs, r,
                       counts, chunk, tk, img);
  else if (tile == 32)
    hipLaunchKernelGGL((k_splat_add<32>), dim3(n_items), dim3(kBlock), 0, s, items, pairs, r,
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

// Persistent launches: as many workgroups as the device holds at once.
template <class K>
static int resident_grid(K kernel, int threads, int n_cu) {
  const int per_cu = cached_occupancy(reinterpret_cast<const void *>(kernel), threads, 0);
  return (per_cu < 1 ? 1 : per_cu) * n_cu;
}

int splat_views_resident(int tile, int n_cu) {
  return tile == 32 ? resident_grid(k_splat_add_views<32>, kBlock, n_cu)
                    : resident_grid(k_splat_add_views<16>, kBlock, n_cu);
}

hipError_t launch_splat_views(int tile, const ViewK *views, const Item *fine, const uint32_t *n_fine,
                              uint32_t *next_fine, const Item *large, const uint32_t *n_large,
                              uint32_t *next_large, int chunk, int cchunk, int n_cu,
                              bool any_large, hipStream_t s) {
  if (any_large)
    hipLaunchKernelGGL(k_splat_large_views,
                       dim3(resident_grid(k_splat_large_views, kLargeThreads, n_cu)),
                       dim3(kLargeThreads), 0, s, views, large, n_large, next_large, cchunk);
  if (tile == 16)
    hipLaunchKernelGGL((k_splat_add_views<16>),
                       dim3(resident_grid(k_splat_add_views<16>, kBlock, n_cu)), dim3(kBlock), 0,
                       s, views, fine, n_fine, next_fine, chunk);
  else if (tile == 32)
    hipLaunchKernelGGL((k_splat_add_views<32>),
                       dim3(resident_grid(k_splat_add_views<32>, kBlock, n_cu)), dim3(kBlock), 0,
                       s, views, fine, n_fine, next_fine, chunk);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_composite(int tile, const Item *items, int n_items,
                            const void *keys, const void *keys_b,
                            uint32_t sort_chunk, const float *rec, const float *rec2,
                            const uint32_t *counts, int chunk, const TileK &tk, float *img,
                            float *partial, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const float4 *r = reinterpret_cast<const float4 *>(rec);
  const float2 *r2 = reinterpret_cast<const float2 *>(rec2);
  float4 *pp = reinterpret_cast<float4 *>(partial);
  const auto *k64 = static_cast<const unsigned long long *>(keys);
  const auto *k64b = static_cast<const unsigned long long *>(keys_b);
  const auto *k32 = static_cast<const uint32_t *>(keys);
  const auto *k32b = static_cast<const uint32_t *>(keys_b);
  auto go = [&](auto kernel, auto ka, auto kb) {
    hipLaunchKernelGGL(kernel, dim3(n_items), dim3(kBlock), 0, s, items, ka, kb, sort_chunk, r, r2,
                       counts, chunk, tk, img, pp);
  };
  // without rec2 (no absorption): the ordered additive sum over index lists
  if (tile == 16)
    r2 ? go(k_composite<16, true>, k64, k64b) : go(k_composite<16, false>, k32, k32b);
  else if (tile == 32)
    r2 ? go(k_composite<32, true>, k64, k64b) : go(k_composite<32, false>, k32, k32b);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_composite_merge(int tile, bool absorb, const Item *items, int n_items,
                                  const uint32_t *counts, int chunk, const TileK &tk,
                                  const float *partial, float *img, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  const float4 *pp = reinterpret_cast<const float4 *>(partial);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(n_items), dim3(kBlock), 0, s, items, counts, chunk, tk, pp,
                       img);
  };
  if (tile == 16)
    absorb ? go(k_composite_merge<16, true>) : go(k_composite_merge<16, false>);
  else if (tile == 32)
    absorb ? go(k_composite_merge<32, true>) : go(k_composite_merge<32, false>);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace spl
