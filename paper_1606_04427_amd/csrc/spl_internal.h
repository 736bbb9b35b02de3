// Internal declarations of the gfx950 Splotch library: kernel parameter
// blocks, launch wrappers and the device helpers that more than one kernel
// must evaluate identically (the single-precision pixel box and tile span).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "splotch.h"

namespace spl {

constexpr int kBlock = 256;
constexpr uint32_t kInactive = 0xffffffffu;
constexpr uint32_t kLargeFlag = 0x80000000u;

// Work item: one chunk of one tile's list.
//   x = bin (tile index), y = first list entry, z = end, w = chunk index.
using Item = uint4;

struct LookK {
  const float *rgb;
  int M;
  int log10;
  int vec;          // 1: colour from the particle's rgb vector
  float beta;
  float lo;
  float inv_range;  // 1/(hi - lo); 0 when hi == lo
};

// Tile geometry of one view.  Fine tiles are bins [0, n_tiles); large-particle
// tiles are bins [n_tiles, n_tiles + n_ctiles).
struct TileK {
  int W, H;
  int tile, ntx, nty, n_tiles;
  int ctile, nctx, ncty, n_ctiles;
  float nu;         // truncation radius in sigma units
  float large_cut;  // px; +inf disables the large path
  int bin_rule;     // 0 exact box, 1 paper distance threshold (fine tiles)
};

struct ProjK {
  // camera frame (FP64)
  double e[3], r[3], u[3], f[3];
  double F, cx, cy, z_near;
  double k_sigma, sigma_min, nu;
  int mode;
  int n_species;
  LookK looks[SPL_MAX_SPECIES];
  // particles
  const float *x, *y, *z;
  const void *h, *inten, *scal;
  int dtype;
  float h_scale, i_scale, s_scale;
  const uint8_t *species;
  const float *absorb;
  const void *rgb;  // colour vectors, 3 per particle (attribute dtype)
  float c_scale;
  int64_t n;
};

// One view of a batch, as the persistent splat kernels read it.
struct ViewK {
  TileK tk;
  const uint32_t *counts;
  const uint32_t *pairs;
  const float4 *rec;
  float *img;
};

// Device totals written by the binning stage and read back by the host.
struct Totals {
  unsigned long long n_active;
  unsigned long long n_large;
  unsigned long long n_pairs;       // all bins
  unsigned long long n_fine_pairs;  // fine bins only
  unsigned long long n_items[3];    // item lists (see build)
  unsigned long long n_fine_items[3];
  unsigned int max_count;           // largest fine-bin count
  unsigned int n_fine_nonempty;     // fine bins with at least one entry
  unsigned int n_coarse_nonempty;   // large-particle bins with at least one entry
  unsigned int pad;
  unsigned long long n_merge_keys;  // keys moved by all merge passes (item list 2)
};

// ---------------------------------------------------------------------------
// Pixel box of a record in single precision.  Each line is one IEEE binary32
// operation, in this order, with contraction disabled: the binning, the
// splat and the host-side checks must all produce the same integers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool record_box(float Xi, float Xf, float Yi, float Yf, float s,
                                           float nu, int W, int H, int &i0, int &i1,
                                           int &j0, int &j1) {
#pragma clang fp contract(off)
  if (!(s > 0.0f)) return false;
  if (!(__builtin_isfinite(Xi) && __builtin_isfinite(Xf) && __builtin_isfinite(Yi) &&
        __builtin_isfinite(Yf) && __builtin_isfinite(s)))
    return false;
  const float R = nu * s;
  const float fx = Xf - 0.5f;
  const float fy = Yf - 0.5f;
  const float lx = fx - R;
  const float hx = fx + R;
  const float ly = fy - R;
  const float hy = fy + R;
  double a0 = (double)Xi + (double)__builtin_ceilf(lx);
  double a1 = (double)Xi + (double)__builtin_floorf(hx);
  double b0 = (double)Yi + (double)__builtin_ceilf(ly);
  double b1 = (double)Yi + (double)__builtin_floorf(hy);
  if (a0 < 0.0) a0 = 0.0;
  if (b0 < 0.0) b0 = 0.0;
  if (a1 > (double)(W - 1)) a1 = (double)(W - 1);
  if (b1 > (double)(H - 1)) b1 = (double)(H - 1);
  if (a0 > a1 || b0 > b1) return false;
  i0 = (int)a0;
  i1 = (int)a1;
  j0 = (int)b0;
  j1 = (int)b1;
  return true;
}

// The paper's tile-inclusion threshold (tile-list pseudocode figure):
// keep tile (tx, ty) if the distance from the particle to the tile centre is
// below 0.75 R + sqrt(2) T / 2.  Single precision, contraction off.
__device__ __forceinline__ bool paper_rule_keeps(float Xi, float Xf, float Yi, float Yf,
                                                 float s, float nu, int tile, int tx, int ty) {
#pragma clang fp contract(off)
  const float R = nu * s;
  const float cx = (float)(tx * tile) + 0.5f * (float)tile;
  const float cy = (float)(ty * tile) + 0.5f * (float)tile;
  const float dx = (Xi - cx) + Xf;
  const float dy = (Yi - cy) + Yf;
  const float t1 = dx * dx;
  const float t2 = dy * dy;
  const float d2 = t1 + t2;
  const float a1 = 0.75f * R;
  const float a2 = (float)tile * 0.70710678f;
  const float thr = a1 + a2;
  const float thr2 = thr * thr;
  return d2 < thr2;
}

// Tile index of pixel v >= 0 for tiles of t > 0 pixels (t is the same on
// every lane: a shift when it is a power of two).
__device__ __forceinline__ uint32_t tile_of(int v, int t) {
  if ((t & (t - 1)) == 0) return (uint32_t)v >> __builtin_ctz((unsigned)t);
  return (uint32_t)v / (uint32_t)t;
}

// Tile span of a record: .x = tx0 | tx1 << 16, .y = ty0 | ty1 << 16, with
// kLargeFlag set in .y when the span is in large-particle tiles.  kInactive in
// .x when the record does not reach the image.
__device__ __forceinline__ uint2 record_span(const float4 r0, float sigma, const TileK &tk) {
  int i0, i1, j0, j1;
  uint2 sp;
  if (!record_box(r0.x, r0.y, r0.z, r0.w, sigma, tk.nu, tk.W, tk.H, i0, i1, j0, j1)) {
    sp.x = kInactive;
    sp.y = kInactive;
    return sp;
  }
  float R;
  {
#pragma clang fp contract(off)
    R = tk.nu * sigma;
  }
  if (R > tk.large_cut) {
    const int c = tk.ctile;
    sp.x = tile_of(i0, c) | (tile_of(i1, c) << 16);
    sp.y = (tile_of(j0, c) | (tile_of(j1, c) << 16)) | kLargeFlag;
  } else {
    const int t = tk.tile;
    sp.x = tile_of(i0, t) | (tile_of(i1, t) << 16);
    sp.y = tile_of(j0, t) | (tile_of(j1, t) << 16);
  }
  return sp;
}

// Merge passes a depth-sorted tile list of c keys takes after the in-LDS
// chunk sorts of k0 keys: runs of k0, 2 k0, 4 k0, ... are merged while they
// are shorter than the list.  Pass i reads buffer i % 2 and writes the other
// one, and a list leaves the passes once it is whole, so it ends in buffer
// merge_passes(c, k0) % 2 (0 = the buffer the scatter wrote).
__host__ __device__ __forceinline__ int merge_passes(uint32_t c, uint32_t k0) {
  int p = 0;
  if (k0 == 0) return 0;
  for (uint64_t L = k0; L < c; L *= 2) ++p;
  return p;
}

// ---------------------------------------------------------------------------
// Launch wrappers (each returns hipSuccess or the launch error).
// ---------------------------------------------------------------------------
// Launches that serve several views of a batch at once (one launch instead of
// one per view: the per-view kernels are small and launch-bound) take up to
// kMaxLaunchViews views, their parameters by value.
constexpr int kMaxLaunchViews = 64;
struct ImgViews {
  float *img[kMaxLaunchViews];
  int64_t n_px[kMaxLaunchViews];
  int blocks[kMaxLaunchViews];  // finalisation blocks of the view
  int aeqe[kMaxLaunchViews];
};
struct ItemViews {
  int nb[kMaxLaunchViews], n_fine[kMaxLaunchViews];
  uint32_t fine[kMaxLaunchViews], coarse[kMaxLaunchViews];  // item array offsets
  uint32_t coarse_shift[kMaxLaunchViews], view[kMaxLaunchViews];
};
// Launch facts of the current device that do not change while the process
// runs, queried once and kept (each HIP query costs microseconds, and the
// launches after a frame's host synchronisation find the device idle until
// they arrive): workgroups of `kernel` a compute unit holds at `threads`
// lanes and `lds` bytes of dynamic LDS (0 if the query fails), and a device
// attribute (0 if the query fails).
int cached_occupancy(const void *kernel, int threads, size_t lds);
int cached_attribute(hipDeviceAttribute_t attr);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
// Copies bytes (a multiple of 4) from device memory into page-locked host
// memory through its device-side address, with a kernel; with flag_mapped
// (the device-side address of a page-locked word), then writes seq there,
// after the copied words are visible to the host.
hipError_t launch_readback(const void *src, void *dst_mapped, size_t bytes, hipStream_t s,
                           void *flag_mapped = nullptr, uint32_t seq = 0);
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
// Zeroes the images iv.img[v] (3 n_px[v] floats) of n_views views.
hipError_t launch_clear_views(const ImgViews &iv, int n_views, hipStream_t s);

// With counts != NULL and project_counts(tk), the projection also adds the
// tile counts of the binning stage into counts (zeroed by the caller).
constexpr int kProjectBins = 8192;
bool project_counts(const TileK &tk);
hipError_t launch_project(const ProjK &pk, const TileK &tk, float *rec, float *rec2,
                          uint2 *span, int write_inactive, Totals *tot, hipStream_t s,
                          uint32_t *counts = nullptr);
// Two additive views of the same particles in one pass (each particle's
// attributes read once), with their tile counts (both project_counts): the
// batch path's pairs of views.  project_pair_ok tells whether two views
// qualify.
bool project_pair_ok(const ProjK &a, const TileK &ta, const ProjK &b, const TileK &tb);
hipError_t launch_project_pair(const ProjK pk[2], const TileK tk[2], float *const rec[2],
                               uint2 *const span[2], Totals *const tot[2],
                               uint32_t *const counts[2], hipStream_t s);
hipError_t launch_span_from_records(const float *rec, int64_t n, const TileK &tk, uint2 *span,
                                    Totals *tot, hipStream_t s);
hipError_t launch_scalar_range(const ProjK &pk, int n_species, int log10, double *out_minmax,
                               hipStream_t s);

// Bin counts from the spans.  umask: ceil(n / kUnitParticles) words the
// count fills with the bands of bins each unit of particles reaches when the
// scatter will need three or more windows of bins (else untouched); pass the
// same buffer to launch_scatter.
constexpr int kUnitParticles = 1024;
hipError_t launch_count(const uint2 *span, const float *rec, int64_t n, const TileK &tk,
                        uint32_t *counts, uint32_t *umask, hipStream_t s);
// Exclusive scan of counts (n_bins) into offsets (n_bins + 1) and cursor; item
// counts for up to three chunk sizes (chunk[k] > 0, powers of two; bins below min_count[k]
// get no item; fine chunk applies to fine bins, cchunk[k] to large bins).
hipError_t launch_scan(const uint32_t *counts, int n_bins, int n_fine, uint32_t *offsets,
                       uint32_t *cursor, const int chunk[3], const int cchunk[3],
                       const int min_count[3], uint32_t *item_off /* 3 x (n_bins+1) */,
                       Totals *tot, hipStream_t s);
// The same for n_views views (host arrays n_bins, n_fine), one workgroup each:
// view v's counts, offsets and cursor start v vstride words after the given
// ones, its item offsets 3 v vstride words after, its totals at tot + v.
hipError_t launch_scan_views(const uint32_t *counts, int n_views, const int *n_bins,
                             const int *n_fine, size_t vstride, uint32_t *offsets,
                             uint32_t *cursor, const int chunk[3], const int cchunk[3],
                             const int min_count[3], uint32_t *item_off, Totals *tot,
                             hipStream_t s);
// Items of fine bins go to items[item_off[b]], items of large bins to
// coarse[item_off[b] - coarse_shift]; the view index is stored in the top 8
// bits of the bin field.
hipError_t launch_build_items(const uint32_t *counts, const uint32_t *offsets, int n_bins,
                              int n_fine, int chunk, int cchunk, int min_count,
                              const uint32_t *item_off, Item *items, hipStream_t s,
                              Item *coarse = nullptr, uint32_t coarse_shift = 0,
                              uint32_t view = 0);
// The same for n_views (<= kMaxLaunchViews) views: view v's counts and
// offsets start v vstride words after the given ones, its item offsets at
// item_off + 3 v vstride + list (nb + 1); its items go to items + iv.fine[v]
// and coarse + iv.coarse[v] (shift iv.coarse_shift[v]), tagged iv.view[v].
hipError_t launch_build_items_views(const uint32_t *counts, const uint32_t *offsets,
                                    size_t vstride, int chunk, int cchunk, int min_count,
                                    const uint32_t *item_off, int list, Item *items, Item *coarse,
                                    const ItemViews &iv, int n_views, hipStream_t s);
hipError_t launch_scatter(const uint2 *span, const float *rec, const float *rec2, int64_t n,
                          const TileK &tk, uint32_t *cursor, uint32_t *pairs,
                          unsigned long long *keys, const uint32_t *umask, hipStream_t s);

// The list sorts take 64-bit (depth bits, index) keys or 32-bit indices (the
// stable order).
hipError_t launch_sort_chunks(unsigned long long *keys, const Item *items, int n_items,
                              hipStream_t s);
hipError_t launch_sort_chunks(uint32_t *keys, const Item *items, int n_items, hipStream_t s);
hipError_t launch_merge_pass(const unsigned long long *src, unsigned long long *dst,
                             const Item *items, int n_items, const uint32_t *offsets,
                             const uint32_t *counts, int run, hipStream_t s);
hipError_t launch_merge_pass(const uint32_t *src, uint32_t *dst, const Item *items, int n_items,
                             const uint32_t *offsets, const uint32_t *counts, int run,
                             hipStream_t s);
hipError_t launch_keys_to_pids(const unsigned long long *keys, int64_t n, uint32_t *pids,
                               hipStream_t s);
// Copies the items of the lists whose merge passes end in the second buffer
// (merge_passes(counts[bin], k0) odd) from src to dst.
hipError_t launch_copy_items(const unsigned long long *src, unsigned long long *dst,
                             const Item *items, int n_items, const uint32_t *counts, uint32_t k0,
                             hipStream_t s);
hipError_t launch_copy_items(const uint32_t *src, uint32_t *dst, const Item *items, int n_items,
                             const uint32_t *counts, uint32_t k0, hipStream_t s);

hipError_t launch_splat_add(int tile, const Item *items, int n_items, const uint32_t *pairs,
                            const float *rec, const uint32_t *counts, int chunk,
                            const TileK &tk, float *img, hipStream_t s);
hipError_t launch_splat_large(const Item *items, int n_items, const uint32_t *pairs,
                              const float *rec, const uint32_t *counts, int cchunk,
                              const TileK &tk, float *img, hipStream_t s);
// Persistent splat over the (view, tile chunk) items of many views: large
// items first, then fine items; n_* and next_* are device counters.
// Workgroups of the persistent additive splat the device holds at once.
int splat_views_resident(int tile, int n_cu);
// any_large: whether the views have large-particle items at all (their
// persistent launch is skipped otherwise).
hipError_t launch_splat_views(int tile, const ViewK *views, const Item *fine, const uint32_t *n_fine,
                              uint32_t *next_fine, const Item *large, const uint32_t *n_large,
                              uint32_t *next_large, int chunk, int cchunk, int n_cu,
                              bool any_large, hipStream_t s);
// keys: the buffer the scatter wrote; keys_b: the merge passes' other buffer
// (each list is read from the one its merge passes end in, sort_chunk = k0).
// With rec2: 64-bit (depth bits, index) keys, the depth-sorted composite,
// which writes img.  rec2 NULL: 32-bit indices in ascending order, no
// absorption, the ordered additive sum, added into img.
hipError_t launch_composite(int tile, const Item *items, int n_items,
                            const void *keys, const void *keys_b,
                            uint32_t sort_chunk, const float *rec, const float *rec2, const uint32_t *counts, int chunk,
                            const TileK &tk, float *img, float *partial, hipStream_t s);
// absorb: as rec2 != NULL in the composite it follows.
hipError_t launch_composite_merge(int tile, bool absorb, const Item *items, int n_items,
                                  const uint32_t *counts, int chunk, const TileK &tk,
                                  const float *partial, float *img, hipStream_t s);

// Resident data sets: largest finite |value x scale| (bits of a
// non-negative float, atomic max into *out_bits), and conversion to the
// stored type (value x sscale x inv_dscale, rounded to nearest even).
hipError_t launch_absmax(const void *src, int dtype, float scale, int64_t n, uint32_t *out_bits,
                         hipStream_t s);
hipError_t launch_convert(const void *src, int sdtype, float sscale, void *dst, int ddtype,
                          float inv_dscale, int64_t n, hipStream_t s);

// Finalisation: kStatPartials FP64 values per block (sums, maxima and sums
// before the map, per channel); the reduction writes stats[0..9] (flux,
// maxima, overall maximum, flux before the map).
constexpr int kStatPartials = 9;
hipError_t launch_finalise(float *img, int64_t n_px, int aeqe, double *partials, int n_blocks,
                           hipStream_t s);
// The same for n_views views (img, n_px, blocks, aeqe of iv), partials of
// view v at partials + v pstride.
hipError_t launch_finalise_views(const ImgViews &iv, int n_views, double *partials,
                                 size_t pstride, hipStream_t s);
// Expected flux sum_p E_p kappa_p of the active records rec[0, n) (span
// not kInactive) into out[0..2]; partials: 3 x n_blocks doubles.
hipError_t launch_expected_flux(const float *rec, const uint2 *span, int64_t n, int W, int H,
                                float nu, double *partials, int n_blocks, double *out,
                                hipStream_t s);
hipError_t launch_reduce_stats(const double *partials, int n_blocks, double *stats,
                               hipStream_t s);
// The same for n_views views (iv.blocks), stats of view v at stats + v sstride.
hipError_t launch_reduce_stats_views(const double *partials, size_t pstride, const ImgViews &iv,
                                     int n_views, double *stats, size_t sstride, hipStream_t s);
hipError_t launch_normalise(float *img, int64_t n_px, const double *stats, hipStream_t s);

}  // namespace spl
