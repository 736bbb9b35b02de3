// Device helpers of the binning stage shared by the kernels that count or
// scatter (particle, tile) pairs: span decoding, run-length aggregation of
// single-tile particles inside a wave, and the hand-out of the pairs of
// multi-tile particles to the whole wave.
#pragma once

#include "spl_internal.h"

namespace spl {

constexpr int kSerialSpan = 16;  // spans of up to this many tiles stay on their lane

struct SpanDec {
  int tx0, tx1, ty0, ty1;
  bool large;
};

__device__ __forceinline__ SpanDec decode(uint2 s) {
  SpanDec d;
  d.tx0 = (int)(s.x & 0xffffu);
  d.tx1 = (int)(s.x >> 16);
  d.ty0 = (int)(s.y & 0xffffu);
  d.ty1 = (int)((s.y >> 16) & 0x7fffu);
  d.large = (s.y & kLargeFlag) != 0;
  return d;
}

// Run-length aggregation inside a wave: consecutive lanes whose particle
// covers exactly one tile, the same one, form a run; the run's first lane
// (head) does one atomic for the whole run.  Returns the run length at the
// head (0 elsewhere); *head_of gets the lane index of the lane's run head.
__device__ __forceinline__ int wave_runs(bool single, int key, int &head_of) {
  const int lane = __lane_id();
  const int prev = __shfl_up(key, 1);
  const bool head = single && (lane == 0 || prev != key);
  const unsigned long long brk = __ballot(!single || head);
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = (lane == 63) ? heads : (heads & ((2ull << lane) - 1ull));
  head_of = upto ? 63 - __builtin_clzll(upto) : lane;
  if (!head) return 0;
  const unsigned long long after = (lane == 63) ? 0ull : (brk >> (lane + 1));
  return after ? (__builtin_ctzll(after) + 1) : (64 - lane);
}

// The (particle, tile) pairs of the wave's multi-tile particles.  A lane
// walks a short span itself; the pairs of long spans are handed out 64 at a
// time to all lanes: the pairs are numbered by a wave prefix sum and
// each lane finds its pair's particle (the owner lane) by a binary search
// over the lanes, so a particle that spans many tiles does not serialise its
// own lane.  For every pair the binning rule keeps, fn(bin, owner_index,
// owner_payload) runs on the lane that took the pair.  Every shuffle runs with
// the whole wave active.
template <class F>
__device__ __forceinline__ void multi_tile_pairs(bool multi, const SpanDec &d, bool filt, int off,
                                                 int ntx, const float4 *__restrict__ rec,
                                                 int64_t k, uint32_t payload, const TileK &tk,
                                                 F &&fn) {
  const int lane = __lane_id();
  const int w = multi ? d.tx1 - d.tx0 + 1 : 1;
  const uint32_t span_tiles = multi ? (uint32_t)(w * (d.ty1 - d.ty0 + 1)) : 0u;
  // the paper rule needs the owner's record; each lane loads its own
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f);
  float sg = 0.f;
  if (filt && multi) {
    r0 = rec[2 * k];
    sg = rec[2 * k + 1].x;
  }
  // short spans: the lane walks its own tiles
  if (span_tiles > 0 && span_tiles <= (uint32_t)kSerialSpan) {
    for (int ty = d.ty0; ty <= d.ty1; ++ty)
      for (int tx = d.tx0; tx <= d.tx1; ++tx)
        if (!filt || paper_rule_keeps(r0.x, r0.y, r0.z, r0.w, sg, tk.nu, tk.tile, tx, ty))
          fn((uint32_t)(off + ty * ntx + tx), (uint32_t)k, payload);
  }
  // long spans: shared by the wave
  const uint32_t cnt = span_tiles > (uint32_t)kSerialSpan ? span_tiles : 0u;
  if (__ballot(cnt != 0u) == 0ull) return;  // uniform
  uint32_t incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = (uint32_t)__shfl_up((int)incl, o);
    if (lane >= o) incl += v;
  }
  const uint32_t total = (uint32_t)__shfl((int)incl, 63);
  const uint32_t excl = incl - cnt;
  const float inv_w = 1.0f / (float)w;
  const bool any_filt = __ballot(filt) != 0ull;
  for (uint32_t r = 0; r < total; r += 64) {  // uniform trip count
    const uint32_t t = r + (uint32_t)lane;
    // owner: the last lane whose first pair number is <= t (lanes without
    // pairs share the first number of the next lane that has some)
    int L = 0;
#pragma unroll
    for (int st = 32; st >= 1; st >>= 1) {
      const uint32_t e = (uint32_t)__shfl((int)excl, L + st);
      if (e <= t) L += st;
    }
    const uint32_t local = t - (uint32_t)__shfl((int)excl, L);
    const uint32_t ow = (uint32_t)__shfl(w, L);
    const float oinv = __shfl(inv_w, L);
    const int otx0 = __shfl(d.tx0, L), oty0 = __shfl(d.ty0, L);
    const int boff = __shfl(off, L), bntx = __shfl(ntx, L);
    const uint32_t ok = (uint32_t)__shfl((int)(uint32_t)k, L);
    const uint32_t opay = (uint32_t)__shfl((int)payload, L);
    uint32_t q = (uint32_t)((float)local * oinv);
    if (q * ow > local)
      --q;
    else if ((q + 1) * ow <= local)
      ++q;
    const int tx = otx0 + (int)(local - q * ow), ty = oty0 + (int)q;
    bool keep = t < total;
    if (any_filt) {
      const bool of = __shfl((int)filt, L) != 0;
      const float x0 = __shfl(r0.x, L), x1 = __shfl(r0.y, L), y0 = __shfl(r0.z, L),
                  y1 = __shfl(r0.w, L), sgo = __shfl(sg, L);
      if (keep && of) keep = paper_rule_keeps(x0, x1, y0, y1, sgo, tk.nu, tk.tile, tx, ty);
    }
    if (keep) fn((uint32_t)(boff + ty * bntx + tx), ok, opay);
  }
}

// Adds one particle's (particle, tile) pairs to the bin counts `bins` (LDS or
// global).  Every lane of the wave must call it; lanes without a particle pass
// an inactive span.  rec is read only for the paper's tile rule.
template <class Add>
__device__ __forceinline__ void count_span_with(uint2 s, int64_t k, const float4 *__restrict__ rec,
                                                const TileK &tk, Add &&add) {
  const bool act = s.x != kInactive;
  const SpanDec d = decode(s);
  const int ntx = d.large ? tk.nctx : tk.ntx;
  const int off = d.large ? tk.n_tiles : 0;
  const bool filt = tk.bin_rule == 1 && !d.large;
  const bool single = act && !filt && d.tx0 == d.tx1 && d.ty0 == d.ty1;
  const int key = single ? off + d.ty0 * ntx + d.tx0 : -1;
  int head_of;
  const int len = wave_runs(single, key, head_of);
  if (len) add((uint32_t)key, (uint32_t)len);
  multi_tile_pairs(act && !single, d, filt, off, ntx, rec, k, 0u, tk,
                   [&](uint32_t bin, uint32_t, uint32_t) { add(bin, 1u); });
}

__device__ __forceinline__ void count_span(uint2 s, int64_t k, const float4 *__restrict__ rec,
                                           const TileK &tk, uint32_t *bins) {
  const bool act = s.x != kInactive;
  const SpanDec d = decode(s);
  const int ntx = d.large ? tk.nctx : tk.ntx;
  const int off = d.large ? tk.n_tiles : 0;
  const bool filt = tk.bin_rule == 1 && !d.large;
  const bool single = act && !filt && d.tx0 == d.tx1 && d.ty0 == d.ty1;
  const int key = single ? off + d.ty0 * ntx + d.tx0 : -1;
  int head_of;
  const int len = wave_runs(single, key, head_of);
  if (len) atomicAdd(&bins[key], (uint32_t)len);
  multi_tile_pairs(act && !single, d, filt, off, ntx, rec, k, 0u, tk,
                   [&](uint32_t bin, uint32_t, uint32_t) { atomicAdd(&bins[bin], 1u); });
}

}  // namespace spl
