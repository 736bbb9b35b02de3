// Tile binning (Sect. 3.1: one particle-index list per tile; tile-list
// pseudocode figure).  The paper grows per-thread dynamic vectors, whose
// allocation it reports as at least half of the Xeon Phi run time
// (Sect. 4.4); here the lists are built without any allocation by
// count -> exclusive scan -> scatter into one preallocated array.
//
//  k_count    per-chunk tile histogram in LDS (global atomics only to flush
//             non-zero bins).  When the bins do not fit in LDS the count and
//             the scatter run once per window of bins that does, each pass
//             over the spans taking the pairs of its window only (a per-pair
//             global atomic, contended on the bins of dense clusters, had
//             taken 17-37 ms at 100M particles and 2048^2 or 4096^2).
//  k_scan     single-workgroup exclusive scan of the bin counts, plus the
//             work-item counts of up to three chunkings of the lists.
//  k_items    expands the item counts into (bin, begin, end, chunk) items.
//  k_scatter  LDS histogram of the workgroup's chunks again, one global
//             atomic per non-zero bin reserves a contiguous range, LDS
//             atomics hand out slots.
#include <algorithm>

#include "bin_device.h"

namespace spl {

namespace {

constexpr int kLdsBins = 16384;  // 64 KB of u32 bins
// Above that a window takes the CU's whole LDS (160 KB on gfx950): one
// 1024-lane workgroup per CU with up to kBigBins u32 bins (scatter) or twice
// as many packed 16-bit bins (count).
constexpr int kBigThreads = 1024;
constexpr int kBigBins = 40960;
constexpr int kChunk = 4096;     // particles per workgroup when the grid is not sized by occupancy

// The count and scatter grids hold no more workgroups than the device keeps
// resident at once (no second, partly filled round), and each workgroup takes
// every gridDim-th unit of kUnit particles: neighbouring indices are often
// neighbours in space, so contiguous shares would hand whole dense clusters
// to a few workgroups, while a unit keeps some neighbours together in each
// tile list (the splat's batches are cheaper when their entries are close).
// unit_block(t) is the first particle of the workgroup's t-th block of 256.
// (NT-lane workgroups take blocks of NT particles.)
constexpr int kUnit = kUnitParticles;
template <int NT = kBlock>
__device__ __forceinline__ int64_t unit_block(int64_t t) {
  constexpr int U = kUnit / NT;
  return ((int64_t)blockIdx.x + (t / U) * (int64_t)gridDim.x) * kUnit + (t % U) * NT;
}

// Whether any (particle, tile) pair of span s can fall in the window of bins
// [lo, lo + nbw): the span's bins lie between its first and last bin.
__device__ __forceinline__ bool span_meets_window(uint2 s, const TileK &tk, int lo, int nbw) {
  if (s.x == kInactive) return false;
  if (lo == 0 && nbw >= tk.n_tiles + tk.n_ctiles) return true;  // one window
  const SpanDec d = decode(s);
  const int ntx = d.large ? tk.nctx : tk.ntx;
  const int off = d.large ? tk.n_tiles : 0;
  const int b0 = off + d.ty0 * ntx + d.tx0, b1 = off + d.ty1 * ntx + d.tx1;
  return b1 >= lo && b0 < lo + nbw;
}

// Unit masks: when the scatter needs three or more windows of bins, the bins are
// also cut into 32 equal bands and each unit of kUnit particles gets the
// bands its particles' pairs can fall in (computed by the first count pass),
// so that a later pass skips, without reading their spans, the units that
// cannot reach its window.
constexpr int kBands = 32;
__host__ __device__ __forceinline__ int band_of_bins(int nb) { return (nb + kBands - 1) / kBands; }
__device__ __forceinline__ uint32_t band_bits(int b0, int b1, int band) {
  const int q0 = b0 / band, q1 = b1 / band;
  return q1 - q0 >= 31 ? (~0u << q0) : (((2u << (q1 - q0)) - 1u) << q0);
}
__device__ __forceinline__ uint32_t span_bands(uint2 s, const TileK &tk, int band) {
  if (s.x == kInactive) return 0u;
  const SpanDec d = decode(s);
  const int ntx = d.large ? tk.nctx : tk.ntx;
  const int off = d.large ? tk.n_tiles : 0;
  return band_bits(off + d.ty0 * ntx + d.tx0, off + d.ty1 * ntx + d.tx1, band);
}
// Whether the unit of particle kb (kb < n) cannot reach the window's bands
// wb (a uniform test: every lane of the workgroup reads the same word).
__device__ __forceinline__ bool unit_skips(const uint32_t *umask, int64_t kb, uint32_t wb) {
  return umask && (umask[kb / kUnit] & wb) == 0u;
}

__global__ __launch_bounds__(kBlock) void k_count(const uint2 *__restrict__ span,
                                                  const float4 *__restrict__ rec, int64_t n,
                                                  TileK tk, uint32_t *__restrict__ counts) {
  extern __shared__ uint32_t hist[];
  const int nb = tk.n_tiles + tk.n_ctiles;
  // the workgroup's histogram covers all its chunks and is flushed once
  for (int i = threadIdx.x; i < nb; i += kBlock) hist[i] = 0;
  __syncthreads();
  {
    int64_t t = 0, kb = unit_block(0);
    // the next span is loaded while this one is counted
    uint2 nxt = (kb + threadIdx.x < n) ? span[kb + threadIdx.x] : make_uint2(kInactive, kInactive);
    while (kb < n) {  // uniform trip count
      const int64_t k = kb + threadIdx.x;
      const int64_t kn = unit_block(++t);
      const uint2 s = nxt;
      nxt = (kn + threadIdx.x < n) ? span[kn + threadIdx.x] : make_uint2(kInactive, kInactive);
      count_span(s, k, rec, tk, hist);
      kb = kn;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    const uint32_t v = hist[i];
    if (v) atomicAdd(&counts[i], v);
  }
}

// The same count with two 16-bit bins per LDS word, so that twice as many
// bins fit (and a workgroup takes half the LDS), over the window of bins
// [lo, lo + nbw).  A bin's count in one workgroup never exceeds the
// particles it takes (a particle adds at most one to a bin), and the grid
// gives no workgroup more than kPackedUnits units, so no half carries into
// the other.
constexpr int kPackedUnits = 63;  // 63 x 1024 particles < 2^16
template <int NT>
__global__ __launch_bounds__(NT) void k_count_packed(const uint2 *__restrict__ span,
                                                         const float4 *__restrict__ rec, int64_t n,
                                                         TileK tk, int lo, int nbw,
                                                         uint32_t *__restrict__ counts,
                                                         uint32_t *__restrict__ umask,
                                                         int make_mask) {
  extern __shared__ uint32_t hist[];
  const int nw = (nbw + 1) / 2;
  // make_mask: this pass builds the unit masks (it reads every span); else a
  // non-null umask lets it skip the units that miss its window
  const int band = band_of_bins(tk.n_tiles + tk.n_ctiles);
  const uint32_t wb = band_bits(lo, lo + nbw - 1, band);
  const uint32_t *skip_mask = make_mask ? nullptr : umask;
  for (int i = threadIdx.x; i < nw; i += NT) hist[i] = 0;
  __syncthreads();
  auto add = [&](uint32_t bin, uint32_t v) {
    const uint32_t b = bin - (uint32_t)lo;  // wraps above the window's top when bin < lo
    if (b < (uint32_t)nbw) atomicAdd(&hist[b >> 1], v << ((b & 1u) * 16u));
  };
  {
    int64_t t = 0, kb = unit_block<NT>(0);
    uint2 nxt = (kb + threadIdx.x < n && !unit_skips(skip_mask, kb, wb))
                    ? span[kb + threadIdx.x]
                    : make_uint2(kInactive, kInactive);
    while (kb < n) {  // uniform trip count
      const int64_t k = kb + threadIdx.x;
      const int64_t kn = unit_block<NT>(++t);
      const uint2 s = nxt;
      nxt = (kn + threadIdx.x < n && !unit_skips(skip_mask, kn, wb))
                ? span[kn + threadIdx.x]
                : make_uint2(kInactive, kInactive);
      if (make_mask) {
        // the bands of the wave's pairs (the wave's particles share a unit)
        uint32_t bits = span_bands(s, tk, band);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) bits |= (uint32_t)__shfl_xor((int)bits, o);
        if (bits && __lane_id() == 0) atomicOr(&umask[kb / kUnit], bits);
      }
      // a wave whose particles all miss the window skips it (uniform)
      if (__ballot(span_meets_window(s, tk, lo, nbw)) != 0ull) count_span_with(s, k, rec, tk, add);
      kb = kn;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nw; i += NT) {
    const uint32_t v = hist[i];
    if (v & 0xffffu) atomicAdd(&counts[lo + 2 * i], v & 0xffffu);
    if (v >> 16) atomicAdd(&counts[lo + 2 * i + 1], v >> 16);
  }
}

// The scatter over the window of bins [lo, lo + nbw): the pairs of other
// bins are left to the window that holds them.
template <bool kKeys, int NT>
__global__ __launch_bounds__(NT) void k_scatter(const uint2 *__restrict__ span,
                                                    const float4 *__restrict__ rec,
                                                    const float2 *__restrict__ rec2, int64_t n,
                                                    TileK tk, int lo, int nbw,
                                                    uint32_t *__restrict__ cursor,
                                                    uint32_t *__restrict__ pairs,
                                                    unsigned long long *__restrict__ keys,
                                                    const uint32_t *__restrict__ umask) {
  extern __shared__ uint32_t hist[];
  // a non-null umask: units whose bands miss the window are skipped unread
  const uint32_t wb = band_bits(lo, lo + nbw - 1, band_of_bins(tk.n_tiles + tk.n_ctiles));
  const bool paper = tk.bin_rule == 1;
  // (wraps above the window's top when bin < lo)
  auto in_win = [&](uint32_t bin) { return bin - (uint32_t)lo < (uint32_t)nbw; };
  // local counts of all the workgroup's chunks, then one global reservation
  // per bin (the order inside a bin is free: additive lists are summed or
  // sorted on the index next, keyed ones are sorted on depth next)
  for (int i = threadIdx.x; i < nbw; i += NT) hist[i] = 0;
  __syncthreads();
  {
    int64_t t = 0, kb = unit_block<NT>(0);
    uint2 nxt = (kb + threadIdx.x < n && !unit_skips(umask, kb, wb))
                    ? span[kb + threadIdx.x]
                    : make_uint2(kInactive, kInactive);
    for (; kb < n; kb = unit_block<NT>(t)) {
      const int64_t k = kb + threadIdx.x;
      const int64_t kn = unit_block<NT>(++t);
      const uint2 s = nxt;
      nxt = (kn + threadIdx.x < n && !unit_skips(umask, kn, wb))
                ? span[kn + threadIdx.x]
                : make_uint2(kInactive, kInactive);
      // a wave whose particles all miss the window skips it (uniform)
      if (__ballot(span_meets_window(s, tk, lo, nbw)) == 0ull) continue;
      const bool act = s.x != kInactive;
      const SpanDec d = decode(s);
      const int ntx = d.large ? tk.nctx : tk.ntx;
      const int off = d.large ? tk.n_tiles : 0;
      const bool filt = paper && !d.large;
      const bool single = act && !filt && d.tx0 == d.tx1 && d.ty0 == d.ty1;
      const int key = single ? off + d.ty0 * ntx + d.tx0 : -1;
      int head_of;
      const int len = wave_runs(single, key, head_of);
      if (len && in_win((uint32_t)key)) atomicAdd(&hist[key - lo], (uint32_t)len);
      multi_tile_pairs(act && !single, d, filt, off, ntx, rec, k, 0u, tk,
                       [&](uint32_t bin, uint32_t, uint32_t) {
                         if (in_win(bin)) atomicAdd(&hist[bin - lo], 1u);
                       });
    }
  }
  __syncthreads();
  // eight bins per lane in flight at once: each reservation returns its
  // base, and one at a time the lane would wait a round trip per bin
  for (int i0 = threadIdx.x; i0 < nbw; i0 += 8 * NT) {
    uint32_t v[8], r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NT;
      v[u] = i < nbw ? hist[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = v[u] ? atomicAdd(&cursor[lo + i0 + u * NT], v[u]) : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u]) hist[i0 + u * NT] = r[u];
  }
  __syncthreads();
  {
    int64_t t = 0, kb = unit_block<NT>(0);
    uint2 nxt = (kb + threadIdx.x < n && !unit_skips(umask, kb, wb))
                    ? span[kb + threadIdx.x]
                    : make_uint2(kInactive, kInactive);
    for (; kb < n; kb = unit_block<NT>(t)) {
      const int64_t k = kb + threadIdx.x;
      const int64_t kn = unit_block<NT>(++t);
      const uint2 s = nxt;
      nxt = (kn + threadIdx.x < n && !unit_skips(umask, kn, wb))
                ? span[kn + threadIdx.x]
                : make_uint2(kInactive, kInactive);
      // a wave whose particles all miss the window skips it (uniform)
      if (__ballot(span_meets_window(s, tk, lo, nbw)) == 0ull) continue;
      const bool act = s.x != kInactive;
      const SpanDec d = decode(s);
      const int ntx = d.large ? tk.nctx : tk.ntx;
      const int off = d.large ? tk.n_tiles : 0;
      const bool filt = paper && !d.large;
      const bool single = act && !filt && d.tx0 == d.tx1 && d.ty0 == d.ty1;
      const int key = single ? off + d.ty0 * ntx + d.tx0 : -1;
      const bool mine = single && in_win((uint32_t)key);
      unsigned long long key_hi = 0;
      if (kKeys && act) key_hi = (unsigned long long)__float_as_uint(rec2[k].y) << 32;
      int head_of;
      const int len = wave_runs(single, key, head_of);
      uint32_t rb = 0;
      if (len && mine) rb = atomicAdd(&hist[key - lo], (uint32_t)len);
      // every lane takes part in the shuffle; run members read their head's base
      const uint32_t hb = (uint32_t)__shfl((int)rb, head_of);
      if (mine) {
        const uint32_t slot = hb + (uint32_t)(__lane_id() - head_of);
        if (kKeys)
          keys[slot] = key_hi | (unsigned long long)(uint32_t)k;
        else
          pairs[slot] = (uint32_t)k;
      }
      multi_tile_pairs(act && !single, d, filt, off, ntx, rec, k, (uint32_t)(key_hi >> 32), tk,
                       [&](uint32_t bin, uint32_t pk, uint32_t zbits) {
                         if (!in_win(bin)) return;
                         const uint32_t slot = atomicAdd(&hist[bin - lo], 1u);
                         if (kKeys)
                           keys[slot] = ((unsigned long long)zbits << 32) | (unsigned long long)pk;
                         else
                           pairs[slot] = pk;
                       });
    }
  }
}

constexpr int kScanThreads = 1024;

// Work items of a bin of c entries in chunks of 2^shift (shift < 0: no
// list; bins below minc entries get none).  Chunk sizes are powers of two.
__device__ __forceinline__ uint32_t items_for(uint32_t c, int bin, int n_fine, int sh, int csh,
                                              int minc) {
  const int shift = bin < n_fine ? sh : csh;
  if (c == 0 || shift < 0 || (int64_t)c < (int64_t)minc) return 0;
  return (c + (1u << shift) - 1u) >> shift;
}

struct ScanArgs {
  int shift[3], cshift[3], minc[3];
};

// Bins and fine bins of each view of one scan launch.
struct ScanViews {
  int nb[kMaxLaunchViews], n_fine[kMaxLaunchViews];
};

// One workgroup: each thread sums a run of consecutive bins (entries and the
// item counts of the three chunkings), the runs are scanned with wave
// shuffles and one pass over the wave totals, and each thread writes its
// bins' offsets.  kLds: the counts are first staged in LDS with coalesced
// loads, so that the threads' runs (consecutive bins per thread) are read
// from LDS rather than with strided global loads, and each output array is
// built in LDS and written with coalesced stores (one workgroup's strided
// stores would otherwise keep a single CU's memory pipeline busy).  LDS
// arrays are padded by one word per 32 so that runs of 2^k bins per thread
// do not fall on one bank.
__device__ __forceinline__ int scan_pad(int b) { return b + (b >> 5); }

// One workgroup per view v = blockIdx.x: the view's arrays start v vstride
// words (item offsets 3 v vstride) after the given ones, its totals at tot + v.
template <bool kLds>
__global__ __launch_bounds__(kScanThreads) void k_scan(const uint32_t *__restrict__ counts0,
                                                       uint32_t *__restrict__ offsets0,
                                                       uint32_t *__restrict__ cursor0, ScanArgs a,
                                                       uint32_t *__restrict__ item_off0,
                                                       Totals *__restrict__ tot0, size_t vstride,
                                                       ScanViews sv) {
  constexpr int NW = kScanThreads / 64;
  const int v = blockIdx.x;
  const int nb = sv.nb[v], n_fine = sv.n_fine[v];
  const uint32_t *__restrict__ counts = counts0 + v * vstride;
  uint32_t *__restrict__ offsets = offsets0 + v * vstride;
  uint32_t *__restrict__ cursor = cursor0 + v * vstride;
  uint32_t *__restrict__ item_off = item_off0 + 3 * v * vstride;
  Totals *__restrict__ tot = tot0 ? tot0 + v : nullptr;
  extern __shared__ uint32_t s_cnt[];
  __shared__ unsigned long long s_w[4][NW];
  __shared__ unsigned int s_max, s_nef, s_nec;
  __shared__ unsigned long long s_l2;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t *const s_pre = s_cnt + scan_pad(nb) + 1;
  auto cnt = [&](int b) { return kLds ? s_cnt[scan_pad(b)] : counts[b]; };
  if (kLds) {
    for (int i = t; i < nb; i += kScanThreads) s_cnt[scan_pad(i)] = counts[i];
    __syncthreads();
  }
  if (t == 0) {
    s_max = 0;
    s_nef = 0;
    s_nec = 0;
    s_l2 = 0;
  }
  const int per = (nb + kScanThreads - 1) / kScanThreads;
  const int b0 = min(t * per, nb), b1 = min(b0 + per, nb);
  unsigned long long loc[4] = {0, 0, 0, 0};
  unsigned int mx = 0, nef = 0, nec = 0;
  unsigned long long l2 = 0;
  for (int b = b0; b < b1; ++b) {
    const uint32_t c = cnt(b);
    loc[0] += c;
    uint32_t ik[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ik[k] = items_for(c, b, n_fine, a.shift[k], a.cshift[k], a.minc[k]);
      loc[1 + k] += ik[k];
    }
    // item list 2 holds the merge-pass items of the lists longer than one
    // chunk sort (min_count[2] - 1 keys): the keys each pass moves
    if (ik[2]) l2 += (unsigned long long)c * (unsigned)merge_passes(c, (uint32_t)(a.minc[2] - 1));
    if (b < n_fine && c > mx) mx = c;
    if (c) {
      if (b < n_fine)
        ++nef;
      else
        ++nec;
    }
  }
  __syncthreads();
  if (mx) atomicMax(&s_max, mx);
  if (nef) atomicAdd(&s_nef, nef);
  if (nec) atomicAdd(&s_nec, nec);
  if (l2) atomicAdd(&s_l2, l2);
  // inclusive scan inside each wave, then over the wave totals
  unsigned long long inc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    inc[q] = loc[q];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long v = __shfl_up(inc[q], o);
      if (lane >= o) inc[q] += v;
    }
    if (lane == 63) s_w[q][wv] = inc[q];
  }
  __syncthreads();
  if (t < 64) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      unsigned long long v = t < NW ? s_w[q][t] : 0ull;
#pragma unroll
      for (int o = 1; o < NW; o <<= 1) {
        const unsigned long long u = __shfl_up(v, o);
        if (t >= o) v += u;
      }
      if (t < NW) s_w[q][t] = v;  // inclusive over waves
    }
  }
  __syncthreads();
  unsigned long long run[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) run[q] = (wv ? s_w[q][wv - 1] : 0ull) + inc[q] - loc[q];
  if (kLds) {
    // one quantity at a time: the run's exclusive prefixes into LDS, then
    // coalesced stores of the whole array
    for (int q = 0; q < 4; ++q) {
      unsigned long long r = run[q];
      for (int b = b0; b < b1; ++b) {
        const uint32_t c = cnt(b);
        if (b == n_fine && tot) {
          if (q == 0)
            tot->n_fine_pairs = r;
          else
            tot->n_fine_items[q - 1] = r;
        }
        s_pre[scan_pad(b)] = (uint32_t)r;
        r += q == 0 ? c : items_for(c, b, n_fine, a.shift[q - 1], a.cshift[q - 1], a.minc[q - 1]);
      }
      __syncthreads();
      if (q == 0) {
        for (int i = t; i < nb; i += kScanThreads) {
          const uint32_t v = s_pre[scan_pad(i)];
          offsets[i] = v;
          cursor[i] = v;
        }
      } else {
        uint32_t *const out = item_off + (q - 1) * (nb + 1);
        for (int i = t; i < nb; i += kScanThreads) out[i] = s_pre[scan_pad(i)];
      }
      __syncthreads();
    }
  } else {
    for (int b = b0; b < b1; ++b) {
      const uint32_t c = cnt(b);
      if (b == n_fine && tot) {
        tot->n_fine_pairs = run[0];
        for (int k = 0; k < 3; ++k) tot->n_fine_items[k] = run[1 + k];
      }
      offsets[b] = (uint32_t)run[0];
      cursor[b] = (uint32_t)run[0];
      run[0] += c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        item_off[k * (nb + 1) + b] = (uint32_t)run[1 + k];
        run[1 + k] += items_for(c, b, n_fine, a.shift[k], a.cshift[k], a.minc[k]);
      }
    }
  }
  if (t == kScanThreads - 1) {
    unsigned long long tt[4];
    for (int q = 0; q < 4; ++q) tt[q] = s_w[q][NW - 1];
    offsets[nb] = (uint32_t)tt[0];
    for (int k = 0; k < 3; ++k) item_off[k * (nb + 1) + nb] = (uint32_t)tt[1 + k];
    if (tot) {
      tot->n_pairs = tt[0];
      for (int k = 0; k < 3; ++k) tot->n_items[k] = tt[1 + k];
      if (n_fine == nb) {
        tot->n_fine_pairs = tt[0];
        for (int k = 0; k < 3; ++k) tot->n_fine_items[k] = tt[1 + k];
      }
      tot->max_count = s_max;
      tot->n_fine_nonempty = s_nef;
      tot->n_coarse_nonempty = s_nec;
      tot->n_merge_keys = s_l2;
    }
  }
}

// View v = blockIdx.y: arrays v vstride words after the given ones (item
// offsets 3 v vstride, then the list `list` of that view's three), items at
// items0 + iv.fine[v], coarse items at coarse0 + iv.coarse[v].
__global__ __launch_bounds__(kBlock) void k_items(const uint32_t *__restrict__ counts0,
                                                  const uint32_t *__restrict__ offsets0,
                                                  int chunk, int cchunk, int minc,
                                                  const uint32_t *__restrict__ item_off0, int list,
                                                  Item *__restrict__ items0,
                                                  Item *__restrict__ coarse0, size_t vstride,
                                                  ItemViews iv) {
  const int v = blockIdx.y;
  const int nb = iv.nb[v], n_fine = iv.n_fine[v];
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b >= nb) return;
  const uint32_t *__restrict__ counts = counts0 + v * vstride;
  const uint32_t *__restrict__ offsets = offsets0 + v * vstride;
  const uint32_t *__restrict__ item_off = item_off0 + 3 * v * vstride + list * (nb + 1);
  Item *__restrict__ items = items0 + iv.fine[v];
  Item *__restrict__ coarse = coarse0 + iv.coarse[v];
  const uint32_t coarse_shift = iv.coarse_shift[v], view = iv.view[v];
  const uint32_t c = counts[b];
  const uint32_t k = items_for(c, b, n_fine, chunk > 0 ? __builtin_ctz((uint32_t)chunk) : -1,
                               cchunk > 0 ? __builtin_ctz((uint32_t)cchunk) : -1, minc);
  if (k == 0) return;
  const uint32_t ch = (uint32_t)(b < n_fine ? chunk : cchunk);
  const uint32_t o = offsets[b], e = o + c;
  Item *dst = (b < n_fine) ? items + item_off[b] : coarse + (item_off[b] - coarse_shift);
  for (uint32_t i = 0; i < k; ++i) {
    const uint32_t s0 = o + i * ch;
    const uint32_t s1 = min(s0 + ch, e);
    dst[i] = make_uint4((uint32_t)b | (view << 24), s0, s1, i);
  }
}

}  // namespace

// Workgroups of the count and scatter passes: as many as the device holds at
// once (each zeroes and flushes a histogram of all bins, and a second, partly
// filled round would cost as much as a full one), at most one per unit of
// kUnit particles.  Without an occupancy figure: one per 4096 particles, fewer when
// there are many bins.
template <typename K>
static int64_t bin_pass_grid(K kernel, size_t sh, int64_t n, int nb, int nt = kBlock) {
  const int64_t units = (n + kUnit - 1) / kUnit;
  const int n_cu = cached_attribute(hipDeviceAttributeMultiprocessorCount);
  const int per_cu = cached_occupancy(reinterpret_cast<const void *>(kernel), nt, sh);
  if (n_cu > 0 && per_cu > 0) return std::min(units, (int64_t)n_cu * per_cu);
  const int64_t cap = nb <= 6144 ? 4096 : (nb <= 12288 ? 2048 : 1024);
  return std::min((n + kChunk - 1) / kChunk, cap);
}

// Windows of the scatter for nb bins: up to kLdsBins bins each while the bins
// fit 64 KB, else up to kBigBins.
static int scatter_windows(int nb) {
  const int cap = nb > kLdsBins ? kBigBins : kLdsBins;
  return (nb + cap - 1) / cap;
}

// Lets a kernel take more than 64 KB of dynamic LDS (a host-side attribute,
// set before each such launch: kernels of one signature share a pointer type).
template <class K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_count(const uint2 *span, const float *rec, int64_t n, const TileK &tk,
                        uint32_t *counts, uint32_t *umask, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = tk.n_tiles + tk.n_ctiles;
  const float4 *r = reinterpret_cast<const float4 *>(rec);
  if (nb <= kLdsBins / 2) {
    const size_t sh = nb * sizeof(uint32_t);
    const int64_t g = bin_pass_grid(k_count, sh, n, nb);
    hipLaunchKernelGGL(k_count, dim3((int)g), dim3(kBlock), sh, s, span, r, n, tk, counts);
    return hipGetLastError();
  }
  // packed 16-bit bins in 1024-lane workgroups: one window up to 2 kLdsBins
  // bins (64 KB, two workgroups per CU; 16384 bins 0.062 -> 0.056 ms at 10M
  // against 512 lanes), else equal windows of at most 2 kBigBins bins in the
  // CU's whole LDS (one pass over the spans each); when the scatter will need
  // three or more windows (where that pays) the first pass also builds the
  // unit masks
  const bool big = nb > 2 * kLdsBins;
  const int cap = big ? 2 * kBigBins : 2 * kLdsBins;
  const int nt = kBigThreads;
  const int n_win = (nb + cap - 1) / cap;
  const int per = (((nb + n_win - 1) / n_win) + 1) & ~1;
  const int64_t units = (n + kUnit - 1) / kUnit;
  if (scatter_windows(nb) < 3) umask = nullptr;
  if (umask) {
    const hipError_t e = launch_fill_u32(umask, 0u, units, s);
    if (e != hipSuccess) return e;
  }
  for (int lo = 0; lo < nb; lo += per) {
    const int nbw = std::min(per, nb - lo);
    const size_t sh = (size_t)((nbw + 1) / 2) * sizeof(uint32_t);
    auto launch = [&](auto kernel) {
      hipError_t e = allow_lds(kernel, sh);
      if (e != hipSuccess) return e;
      const int64_t g =
          std::max(bin_pass_grid(kernel, sh, n, nbw, nt), (units + kPackedUnits - 1) / kPackedUnits);
      hipLaunchKernelGGL(kernel, dim3((int)g), dim3(nt), sh, s, span, r, n, tk, lo, nbw, counts,
                         umask, (int)(lo == 0 && umask != nullptr));
      return hipGetLastError();
    };
    const hipError_t e = launch(k_count_packed<kBigThreads>);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scan_views(const uint32_t *counts, int n_views, const int *n_bins,
                             const int *n_fine, size_t vstride, uint32_t *offsets,
                             uint32_t *cursor, const int chunk[3], const int cchunk[3],
                             const int min_count[3], uint32_t *item_off, Totals *tot,
                             hipStream_t s) {
  ScanArgs a;
  auto shift_of = [](int ch) {
    if (ch <= 0) return -1;
    int sft = 0;
    while ((1 << sft) < ch) ++sft;
    return sft;
  };
  for (int k = 0; k < 3; ++k) {
    if ((chunk[k] > 0 && (chunk[k] & (chunk[k] - 1))) || (cchunk[k] > 0 && (cchunk[k] & (cchunk[k] - 1))))
      return hipErrorInvalidValue;  // chunk sizes are powers of two
    a.shift[k] = shift_of(chunk[k]);
    a.cshift[k] = shift_of(cchunk[k]);
    a.minc[k] = min_count[k];
  }
  // counts and one output array are staged in LDS when they fit beside the
  // kernel's own 1 KB
  const int lds_max = cached_attribute(hipDeviceAttributeMaxSharedMemoryPerBlock);
  // views in launches of up to kMaxLaunchViews workgroups
  for (int v0 = 0; v0 < n_views; v0 += kMaxLaunchViews) {
    const int nv = std::min(kMaxLaunchViews, n_views - v0);
    ScanViews sv;
    int max_bins = 0;
    for (int v = 0; v < nv; ++v) {
      sv.nb[v] = n_bins[v0 + v];
      sv.n_fine[v] = n_fine[v0 + v];
      max_bins = std::max(max_bins, sv.nb[v]);
    }
    const size_t o = (size_t)v0 * vstride;
    Totals *t = tot ? tot + v0 : nullptr;
    const int64_t lds = 2 * ((int64_t)max_bins + max_bins / 32 + 1) * (int64_t)sizeof(uint32_t);
    if (lds + 1024 <= (int64_t)lds_max)
      hipLaunchKernelGGL(k_scan<true>, dim3(nv), dim3(kScanThreads), (size_t)lds, s, counts + o,
                         offsets + o, cursor + o, a, item_off + 3 * o, t, vstride, sv);
    else
      hipLaunchKernelGGL(k_scan<false>, dim3(nv), dim3(kScanThreads), 0, s, counts + o,
                         offsets + o, cursor + o, a, item_off + 3 * o, t, vstride, sv);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_scan(const uint32_t *counts, int n_bins, int n_fine, uint32_t *offsets,
                       uint32_t *cursor, const int chunk[3], const int cchunk[3],
                       const int min_count[3], uint32_t *item_off, Totals *tot, hipStream_t s) {
  return launch_scan_views(counts, 1, &n_bins, &n_fine, 0, offsets, cursor, chunk, cchunk,
                           min_count, item_off, tot, s);
}

hipError_t launch_build_items_views(const uint32_t *counts, const uint32_t *offsets,
                                    size_t vstride, int chunk, int cchunk, int min_count,
                                    const uint32_t *item_off, int list, Item *items, Item *coarse,
                                    const ItemViews &iv, int n_views, hipStream_t s) {
  if (n_views < 1 || n_views > kMaxLaunchViews) return hipErrorInvalidValue;
  int max_bins = 0;
  for (int v = 0; v < n_views; ++v) max_bins = std::max(max_bins, iv.nb[v]);
  if (max_bins == 0) return hipSuccess;
  const int g = (max_bins + kBlock - 1) / kBlock;
  if (!coarse) coarse = items;
  hipLaunchKernelGGL(k_items, dim3(g, n_views), dim3(kBlock), 0, s, counts, offsets, chunk,
                     cchunk, min_count, item_off, list, items, coarse, vstride, iv);
  return hipGetLastError();
}

hipError_t launch_build_items(const uint32_t *counts, const uint32_t *offsets, int n_bins,
                              int n_fine, int chunk, int cchunk, int min_count,
                              const uint32_t *item_off, Item *items, hipStream_t s, Item *coarse,
                              uint32_t coarse_shift, uint32_t view) {
  ItemViews iv;
  iv.nb[0] = n_bins;
  iv.n_fine[0] = n_fine;
  iv.fine[0] = 0;
  iv.coarse[0] = 0;
  iv.coarse_shift[0] = coarse_shift;
  iv.view[0] = view;
  return launch_build_items_views(counts, offsets, 0, chunk, cchunk, min_count, item_off, 0,
                                  items, coarse, iv, 1, s);
}

hipError_t launch_scatter(const uint2 *span, const float *rec, const float *rec2, int64_t n,
                          const TileK &tk, uint32_t *cursor, uint32_t *pairs,
                          unsigned long long *keys, const uint32_t *umask, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = tk.n_tiles + tk.n_ctiles;
  const float4 *r = reinterpret_cast<const float4 *>(rec);
  const float2 *r2 = reinterpret_cast<const float2 *>(rec2);
  // equal windows (one launch, two passes over the spans, each)
  const int n_win = scatter_windows(nb);
  const int per = (nb + n_win - 1) / n_win;
  if (n_win < 3) umask = nullptr;  // (built by the count from three windows on)
  for (int lo = 0; lo < nb; lo += per) {
    const int nbw = std::min(per, nb - lo);
    const size_t sh = (size_t)nbw * sizeof(uint32_t);
    auto launch = [&](auto kernel, int nt) {
      hipError_t e = allow_lds(kernel, sh);
      if (e != hipSuccess) return e;
      const int64_t g = bin_pass_grid(kernel, sh, n, nbw, nt);
      hipLaunchKernelGGL(kernel, dim3((int)g), dim3(nt), sh, s, span, r, r2, n, tk, lo, nbw, cursor,
                         pairs, keys, umask);
      return hipGetLastError();
    };
    // 1024-lane workgroups in every window: two per CU up to 64 KB of bins,
    // one above.  Each workgroup reserves its slots with one global atomic
    // per non-empty bin, so fewer, wider workgroups issue fewer of them (10M
    // particles: 4352 bins 0.108 -> 0.100 ms per view against 256-lane
    // workgroups, 16384 bins 0.196 -> 0.153 ms against 512 lanes; one
    // 1024-lane workgroup per CU was slower than two, 0.136 ms at 4352 bins)
    const hipError_t e = keys ? launch(k_scatter<true, kBigThreads>, kBigThreads)
                              : launch(k_scatter<false, kBigThreads>, kBigThreads);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace spl
