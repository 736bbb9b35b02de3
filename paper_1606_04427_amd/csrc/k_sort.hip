// Depth ordering of the tile lists for the non-additive transfer mode
// (Sect. 2.1: the transfer equation makes compositing order-dependent).
// Keys are 64-bit: the IEEE bits of the (positive) view depth in the high
// word and the particle index in the low word, so ascending keys are
// ascending (depth, index) and every key is unique.  The same kernels sort
// 32-bit keys, the particle indices alone, for the lists in ascending index
// (the stable order of the additive frames drawn in list order).
//
//  k_sort_chunks  one workgroup per list chunk of <= 4096 keys: bitonic sort
//                 with up to 8 keys per lane of 512 in registers.  A list
//                 that fits one chunk is done.
//  k_merge_pass   longer lists: sorted runs of length L merged pairwise into
//                 runs of 2L; one workgroup per 2048 outputs stages its inputs
//                 in LDS, each lane merges 8 keys into LDS, and the outputs
//                 leave with coalesced stores.  A list that is whole skips
//                 the remaining passes (merge_passes gives its buffer).
#include "spl_internal.h"

namespace spl {

namespace {

constexpr int kSortChunk = 4096;
constexpr int kMergeOut = 2048;  // outputs per workgroup = 256 lanes x 8

__device__ __forceinline__ int padded(int pos) { return pos + (pos >> 4); }

// Compare-exchange stage with partners J < E apart inside one thread's keys.
template <int J, int E, typename K>
__device__ __forceinline__ void reg_stage(K (&v)[E], int t, int k) {
  if constexpr (J < E) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if ((e & J) == 0) {
        // ascending pairs swap when b < a, descending ones when not (equal
        // keys are only padding, so swapping them changes nothing)
        const bool up = ((t * E + e) & k) == 0;
        const K a = v[e], b = v[e + J];
        const bool sw = (b < a) == up;
        v[e] = sw ? b : a;
        v[e + J] = sw ? a : b;
      }
    }
  }
}

// Partner key of lane ^ m for m < 32: DPP lane permutes inside quads for
// m = 1, 2, LDS swizzles (no address operand) otherwise.
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  if constexpr (M == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xf, 0xf, false);
  } else if constexpr (M == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xf, 0xf, false);
  } else {
    constexpr int pat = 0x1f | (M << 10);  // bit-mask mode: and 31, xor M
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, pat);
  }
}
template <int M>
__device__ __forceinline__ unsigned long long xor_lane(unsigned long long v) {
  const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  int a, b;
  if constexpr (M == 1) {
    a = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xf, 0xf, false);
    b = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xf, 0xf, false);
  } else if constexpr (M == 2) {
    a = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xf, 0xf, false);
    b = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xf, 0xf, false);
  } else {
    constexpr int pat = 0x1f | (M << 10);  // bit-mask mode: and 31, xor M
    a = __builtin_amdgcn_ds_swizzle(lo, pat);
    b = __builtin_amdgcn_ds_swizzle(hi, pat);
  }
  return (unsigned long long)(uint32_t)a | ((unsigned long long)(uint32_t)b << 32);
}

// Bitonic sort of one chunk of np = NT E keys (padded with ~0): thread t
// holds the E consecutive keys t E .. t E + E - 1 in registers.  Compare-
// exchange partners closer than E sit in the same thread; partners up to
// 64 E away sit in the same wave and are read with a lane shuffle; farther
// ones go through LDS.  Loads and stores pass through LDS so that global
// accesses stay coalesced.
template <int E, int NT, typename K>
__device__ __forceinline__ void sort_chunk(K *__restrict__ keys, uint32_t b0, int n, K *s) {
  constexpr int NP = NT * E;
  const int t = threadIdx.x;
  for (int p = t; p < NP; p += NT) s[padded(p)] = (p < n) ? keys[b0 + p] : ~(K)0;
  __syncthreads();
  K v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = s[padded(t * E + e)];
#pragma unroll 1
  for (int k = 2; k <= NP; k <<= 1) {
#pragma unroll 1
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < E) {
        switch (j) {
          case 1: reg_stage<1, E>(v, t, k); break;
          case 2: reg_stage<2, E>(v, t, k); break;
          case 4: reg_stage<4, E>(v, t, k); break;
          default: reg_stage<8, E>(v, t, k); break;
        }
      } else {
        const int m = j / E;  // partner thread: t ^ m
        // j >= E and k > j: whether the lane keeps the smaller key does not
        // depend on e
        const bool keep_min = ((t * E & j) == 0) == ((t * E & k) == 0);
        if (m < 64) {
          auto cx = [&](auto partner) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
              const K w = partner(v[e]);
              v[e] = ((w < v[e]) == keep_min) ? w : v[e];
            }
          };
          switch (m) {
            case 1: cx([](K x) { return xor_lane<1>(x); }); break;
            case 2: cx([](K x) { return xor_lane<2>(x); }); break;
            case 4: cx([](K x) { return xor_lane<4>(x); }); break;
            case 8: cx([](K x) { return xor_lane<8>(x); }); break;
            case 16: cx([](K x) { return xor_lane<16>(x); }); break;
            default: cx([](K x) { return __shfl_xor(x, 32); }); break;
          }
        } else {
          __syncthreads();
#pragma unroll
          for (int e = 0; e < E; ++e) s[padded(t * E + e)] = v[e];
          __syncthreads();
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const K w = s[padded((t ^ m) * E + e)];
            v[e] = ((w < v[e]) == keep_min) ? w : v[e];
          }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) s[padded(t * E + e)] = v[e];
  __syncthreads();
  for (int p = t; p < n; p += NT) keys[b0 + p] = s[padded(p)];
}

// 512 lanes per workgroup, up to 8 keys each: the 34 KB of LDS allow four
// workgroups per CU, and 512-lane ones bring twice the waves of 256-lane
// ones (at the price of one more stage through LDS per merge level).
constexpr int kSortThreads = 512;
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_chunks(K *__restrict__ keys,
                                                              const Item *__restrict__ items) {
  constexpr int NT = kSortThreads;
  static_assert(NT * 8 == kSortChunk, "a chunk is 8 keys per lane");
  __shared__ K s[kSortChunk + kSortChunk / 16];
  const Item it = items[blockIdx.x];
  const int n = (int)(it.z - it.y);
  if (n <= NT)
    sort_chunk<1, NT>(keys, it.y, n, s);
  else if (n <= 2 * NT)
    sort_chunk<2, NT>(keys, it.y, n, s);
  else if (n <= 4 * NT)
    sort_chunk<4, NT>(keys, it.y, n, s);
  else
    sort_chunk<8, NT>(keys, it.y, n, s);
}

// First i in [lo, hi) with A[i] >= B[diag - 1 - i] (hi if none): the start
// of the merge path's crossing of diagonal `diag`.  One wave tests 64 evenly
// spaced candidates per round and keeps the bracket where the predicate turns,
// so a search over L candidates takes log64(L) rounds of global loads.
template <typename K>
__device__ __forceinline__ int64_t wave_merge_split(const K *__restrict__ A,
                                                    const K *__restrict__ B,
                                                    int64_t diag, int64_t lo, int64_t hi) {
  const int lane = __lane_id();
  while (hi > lo) {  // uniform across the wave
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t i = lo + (int64_t)lane * step;
    const bool p = i < hi && A[i] < B[diag - 1 - i];
    const int c = __popcll(__ballot(p));  // the true candidates form a prefix
    if (c == 0) {
      hi = lo;
    } else {
      const int64_t nlo = lo + (int64_t)(c - 1) * step + 1;
      hi = min(hi, lo + (int64_t)c * step);
      lo = nlo;
    }
  }
  return lo;
}

// One merge pass: sorted runs of length L merged pairwise into runs of 2L.
// A workgroup owns kMergeOut consecutive outputs of one list (they fall in one
// pair of runs because 2L is a multiple of kMergeOut).  Waves 0 and 1 find
// where the merge path enters and leaves that output range, the inputs
// between are staged in LDS with coalesced loads, each lane merges 8
// outputs from LDS after a binary search there, and the merged range is
// written back with coalesced stores.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_merge_pass(const K *__restrict__ src,
                                                       K *__restrict__ dst,
                                                       const Item *__restrict__ items,
                                                       const uint32_t *__restrict__ offsets,
                                                       const uint32_t *__restrict__ counts,
                                                       int64_t L) {
  __shared__ K s_k[kMergeOut];
  __shared__ K s_o[kMergeOut];  // merged outputs, stored coalesced
  __shared__ int64_t s_split[2];
  const Item it = items[blockIdx.x];
  const int64_t s0 = offsets[it.x];
  const int64_t n = counts[it.x];
  // a list no longer than L is whole already and stays where it is
  if (n <= L) return;
  const int64_t d0 = (int64_t)it.y - s0, d1 = (int64_t)it.z - s0;
  const int64_t ps = (d0 / (2 * L)) * (2 * L);
  const int64_t la = min(L, n - ps);
  const int64_t lb = max((int64_t)0, min(L, n - ps - L));
  const K *A = src + s0 + ps;
  const K *B = A + L;
  const int wave = threadIdx.x >> 6;
  if (wave < 2) {
    const int64_t diag = (wave == 0 ? d0 : d1) - ps;
    const int64_t a = wave_merge_split(A, B, diag, max((int64_t)0, diag - lb), min(diag, la));
    if (__lane_id() == 0) s_split[wave] = a;
  }
  __syncthreads();
  const int64_t a0 = s_split[0], a1 = s_split[1];
  const int64_t b0 = (d0 - ps) - a0, b1 = (d1 - ps) - a1;
  const int na = (int)(a1 - a0), nb = (int)(b1 - b0);
  for (int i = threadIdx.x; i < na; i += kBlock) s_k[i] = A[a0 + i];
  for (int i = threadIdx.x; i < nb; i += kBlock) s_k[na + i] = B[b0 + i];
  __syncthreads();
  const int tot = na + nb;
  const int dl = 8 * (int)threadIdx.x;
  if (dl < tot) {
    const K *As = s_k, *Bs = s_k + na;
    int lo = max(0, dl - nb), hi = min(dl, na);
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (As[mid] < Bs[dl - 1 - mid])
        lo = mid + 1;
      else
        hi = mid;
    }
    int i = lo, j = dl - lo;
    const int cnt = min(8, tot - dl);
    for (int o = 0; o < cnt; ++o) {
      K v;
      if (j >= nb || (i < na && As[i] < Bs[j]))
        v = As[i++];
      else
        v = Bs[j++];
      s_o[dl + o] = v;
    }
  }
  __syncthreads();
  K *out = dst + s0 + d0;
  for (int k = threadIdx.x; k < tot; k += kBlock) out[k] = s_o[k];
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_copy_items(const K *__restrict__ src,
                                                       K *__restrict__ dst,
                                                       const Item *__restrict__ items,
                                                       const uint32_t *__restrict__ counts,
                                                       uint32_t k0) {
  const Item it = items[blockIdx.x];
  if ((merge_passes(counts[it.x], k0) & 1) == 0) return;
  for (uint32_t k = it.y + threadIdx.x; k < it.z; k += kBlock) dst[k] = src[k];
}

__global__ __launch_bounds__(kBlock) void k_keys_to_pids(const unsigned long long *__restrict__ keys,
                                                         int64_t n, uint32_t *__restrict__ pids) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    pids[i] = (uint32_t)(keys[i] & 0xffffffffull);
}

}  // namespace

hipError_t launch_keys_to_pids(const unsigned long long *keys, int64_t n, uint32_t *pids,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_keys_to_pids, dim3((int)g), dim3(kBlock), 0, s, keys, n, pids);
  return hipGetLastError();
}

template <typename K>
static hipError_t sort_chunks(K *keys, const Item *items, int n_items, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_chunks<K>, dim3(n_items), dim3(kSortThreads), 0, s, keys, items);
  return hipGetLastError();
}

template <typename K>
static hipError_t merge_pass(const K *src, K *dst, const Item *items, int n_items,
                             const uint32_t *offsets, const uint32_t *counts, int run,
                             hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_pass<K>, dim3(n_items), dim3(kBlock), 0, s, src, dst, items, offsets,
                     counts, (int64_t)run);
  return hipGetLastError();
}

template <typename K>
static hipError_t copy_items(const K *src, K *dst, const Item *items, int n_items,
                             const uint32_t *counts, uint32_t k0, hipStream_t s) {
  if (n_items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_items<K>, dim3(n_items), dim3(kBlock), 0, s, src, dst, items, counts,
                     k0);
  return hipGetLastError();
}

hipError_t launch_sort_chunks(unsigned long long *keys, const Item *items, int n_items,
                              hipStream_t s) {
  return sort_chunks(keys, items, n_items, s);
}
hipError_t launch_sort_chunks(uint32_t *keys, const Item *items, int n_items, hipStream_t s) {
  return sort_chunks(keys, items, n_items, s);
}

hipError_t launch_merge_pass(const unsigned long long *src, unsigned long long *dst,
                             const Item *items, int n_items, const uint32_t *offsets,
                             const uint32_t *counts, int run, hipStream_t s) {
  return merge_pass(src, dst, items, n_items, offsets, counts, run, s);
}
hipError_t launch_merge_pass(const uint32_t *src, uint32_t *dst, const Item *items, int n_items,
                             const uint32_t *offsets, const uint32_t *counts, int run,
                             hipStream_t s) {
  return merge_pass(src, dst, items, n_items, offsets, counts, run, s);
}

hipError_t launch_copy_items(const unsigned long long *src, unsigned long long *dst,
                             const Item *items, int n_items, const uint32_t *counts, uint32_t k0,
                             hipStream_t s) {
  return copy_items(src, dst, items, n_items, counts, k0, s);
}
hipError_t launch_copy_items(const uint32_t *src, uint32_t *dst, const Item *items, int n_items,
                             const uint32_t *counts, uint32_t k0, hipStream_t s) {
  return copy_items(src, dst, items, n_items, counts, k0, s);
}

}  // namespace spl
