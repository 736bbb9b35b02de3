// C ABI of the gfx950 Splotch library: argument checks, the context
// workspace, and the order of kernel launches for one frame.
//
// Frame (Sect. 2.1 rasterisation + rendering; Sect. 3.1 tiles):
//   project+colour (+ tile counts when the bins fit LDS) [-> count] -> scan
//   [one stream sync: list sizes]
//   -> build work items -> scatter -> (sort) -> splat / composite
//   -> finalise (+ FP64 flux / max) [-> normalise]
// The single host synchronisation per frame reads the list sizes so that
// every list and item buffer is sized exactly; no kernel can overflow a
// buffer.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "spl_internal.h"

using namespace spl;

// Workspace of spl_render_noalloc: one copy per device, held until the
// process ends.  Host code never passes this name to a kernel; it uses the
// device address that spl_create looks up for each device.
constexpr size_t kScratchBytes = (size_t)128 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kChunkSplat = 1024;  // list entries per splat item, fine tiles
constexpr int kChunkLarge = 512;   // list entries per large-particle item
// List entries per splat item in the batch path when the batch holds enough
// work: items four times longer still keep every slot of the device busy,
// and a dense tile is then merged from a quarter as many partial results
// (float atomics on the image).  A batch with fewer long items than
// kViewsItemsPerSlot per resident workgroup keeps the shorter items, which
// balance better.  The scan counts the items of both lengths.
constexpr int kChunkViews = 4096;
constexpr int kViewsItemsPerSlot = 8;
constexpr int kSortChunk = 4096;   // keys per in-LDS sort
constexpr int kMergeOut = 2048;    // outputs per merge workgroup
constexpr int kLargeTile = 64;     // px, tiles of the large-particle path
constexpr int kDefaultTile = 16;
constexpr double kDefaultCut = 32.0;  // px
constexpr int kFinBlocks = 1024;
// FP64 statistics per view: [0..2] flux, [3..5] max, [6] overall max,
// [7..9] flux before the map, [10..12] expected flux
constexpr int kStatWords = 16;

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
};

// A fixed region that ensure() carves buffers from instead of allocating.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

constexpr int kMaxDevices = 64;
std::mutex g_launch_mu;  // guards the two caches below
std::map<std::tuple<int, const void *, int, size_t>, int> g_occupancy;
std::map<std::pair<int, int>, int> g_attribute;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// Events of one timed frame: ev[k] .. ev[k+1] brackets stage k.
struct TimedFrame {
  hipEvent_t ev[SPL_N_STAGES + 1];
  double bytes[SPL_N_STAGES];
  int frames = 1;  // views the events cover (a batch covers several)
};

}  // namespace

namespace spl {

int cached_occupancy(const void *kernel, int threads, size_t lds) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const auto key = std::make_tuple(dev, kernel, threads, lds);
  {
    std::lock_guard<std::mutex> lk(g_launch_mu);
    auto it = g_occupancy.find(key);
    if (it != g_occupancy.end()) return it->second;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;  // not kept: a later call asks again
  }
  std::lock_guard<std::mutex> lk(g_launch_mu);
  g_occupancy[key] = per_cu;
  return per_cu;
}

int cached_attribute(hipDeviceAttribute_t attr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const auto key = std::make_pair(dev, (int)attr);
  {
    std::lock_guard<std::mutex> lk(g_launch_mu);
    auto it = g_attribute.find(key);
    if (it != g_attribute.end()) return it->second;
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, attr, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> lk(g_launch_mu);
  g_attribute[key] = v;
  return v;
}

}  // namespace spl

// A resident particle set: one device allocation holding every array.
struct spl_dataset {
  int device = 0;
  spl_particles view{};  // device pointers into mem, stored dtype and scales
  void *mem = nullptr;
  size_t bytes = 0;
};

struct spl_ctx {
  int device = 0;
  std::string err;
  DevBuf rec, rec2, span, counts, offsets, cursor, item_off, items[3], pairs, keysA, keysB,
      partial, fin, stats, totals, minmax, himg, chunk[2];
  DevBuf umask;  // bands of bins per unit of particles (binning in windows)
  hipStream_t copy_stream = nullptr;  // host-to-device copies of spl_render_stream
  hipEvent_t ev_copied[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
  Totals *h_tot = nullptr;   // page-locked host memory ...
  double *h_stats = nullptr;
  void *m_tot = nullptr;     // ... and its device-side addresses, written by
  void *m_stats = nullptr;   // the read-back kernel
  // read-back completion word (page-locked, device-side address m_flag): the
  // read-back kernel writes the call's sequence number there after the data
  uint32_t *h_flag = nullptr;
  void *m_flag = nullptr;
  uint32_t rb_seq = 0;
  int64_t bytes = 0;
  // autotuner choices: per (n, W, H, mode, camera pose), and the most
  // recent choice per (n, W, H, mode) for poses that were not tuned
  std::map<std::tuple<int64_t, int, int, int, uint64_t>, std::pair<int, double>> tune;
  std::map<std::tuple<int64_t, int, int, int>, std::pair<int, double>> tune_any;
  // stage timers
  bool timing = false;
  std::vector<hipEvent_t> event_pool;
  std::vector<TimedFrame> pending;
  double acc_ms[SPL_N_STAGES] = {0};
  double acc_bytes[SPL_N_STAGES] = {0};
  int64_t acc_frames = 0;
  // many-view batches
  DevBuf b_rec, b_span, b_counts, b_offsets, b_cursor, b_itemoff, b_totals, b_pairs, b_itf,
      b_itc, b_views, b_ctr, b_fin, b_stats, b_umask;
  Totals *h_btot = nullptr;
  ViewK *h_views = nullptr;
  uint32_t *h_ctr = nullptr;
  double *h_bstats = nullptr;
  void *m_btot = nullptr, *m_bstats = nullptr;  // device-side addresses
  int h_cap = 0;  // views the pinned host arrays hold
  bool graphs = false;
  hipStream_t cap_stream = nullptr;   // capture stream for batch graphs
  hipGraphExec_t gexec = nullptr;     // last instantiated batch graph
  int64_t budget = (int64_t)48 << 30;
  uint64_t group_pairs = 0xfffffffeull;  // list entries per persistent launch
  int n_cu = 256;
  void *scratch = nullptr;  // this device's copy of `scratch`
  Arena *arena = nullptr;   // set while spl_render_noalloc runs
};

namespace {

// Page-locked host memory that the read-back kernel writes while the host
// watches it: fine-grained (coherent), so the device's stores go to host
// memory instead of waiting in a device cache for a write-back; the default
// (coarse-grained) kind if the runtime refuses that.
hipError_t watched_host_alloc(void **p, size_t bytes) {
  if (hipHostMalloc(p, bytes, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess)
    return hipSuccess;
  (void)hipGetLastError();
  *p = nullptr;
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

spl_status fail(spl_ctx *c, spl_status code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
spl_status fail(spl_ctx *c, spl_status code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIPTRY(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((ctx), SPL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

spl_status ensure(spl_ctx *c, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.cap >= bytes) return SPL_OK;
  if (c->arena) {
    Arena &a = *c->arena;
    const size_t off = (a.used + 255) & ~(size_t)255;
    if (off > a.cap || bytes > a.cap - off)
      return fail(c, SPL_ENOMEM,
                  "the %zu-byte scratch cannot hold this frame: %zu more bytes needed with %zu "
                  "in use",
                  a.cap, bytes, off);
    b.p = a.base + off;
    b.cap = bytes;
    a.used = off + bytes;
    return SPL_OK;
  }
  size_t want = b.cap + b.cap / 2;
  if (want < bytes) want = bytes;
  want = (want + 255) & ~(size_t)255;
  if (b.p) {
    (void)hipFree(b.p);
    c->bytes -= (int64_t)b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      b.p = nullptr;
      (void)hipGetLastError();
      return fail(c, SPL_ENOMEM, "device allocation of %zu bytes failed", bytes);
    }
    want = bytes;
  }
  b.cap = want;
  c->bytes += (int64_t)want;
  return SPL_OK;
}

#define TRY(expr)                  \
  do {                             \
    spl_status r_ = (expr);        \
    if (r_ != SPL_OK) return r_;   \
  } while (0)

bool finite3(const double *v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

// Camera frame: forward f = (lookat - eye)/|..|, right r = f x up/|..|,
// up' = r x f, focal length F = (H/2)/tan(fov/2).
spl_status camera_frame(spl_ctx *c, const spl_camera *cam, ProjK &pk) {
  if (!cam) return fail(c, SPL_EINVAL, "camera is NULL");
  if (cam->width < 1 || cam->height < 1 || cam->width > 32768 || cam->height > 32768)
    return fail(c, SPL_EINVAL, "image size %dx%d outside 1..32768", cam->width, cam->height);
  if (!(cam->fov_y_deg > 0.0 && cam->fov_y_deg < 180.0))
    return fail(c, SPL_EINVAL, "fov_y_deg %g outside (0, 180)", cam->fov_y_deg);
  if (!(cam->z_near >= 0.0) || !std::isfinite(cam->z_near))
    return fail(c, SPL_EINVAL, "z_near must be finite and >= 0");
  if (!finite3(cam->eye) || !finite3(cam->lookat) || !finite3(cam->up))
    return fail(c, SPL_EINVAL, "camera vectors must be finite");
  double f[3], r[3], u[3];
  for (int k = 0; k < 3; ++k) f[k] = cam->lookat[k] - cam->eye[k];
  double nf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(nf > 0.0)) return fail(c, SPL_EINVAL, "eye and lookat coincide");
  for (double &v : f) v /= nf;
  r[0] = f[1] * cam->up[2] - f[2] * cam->up[1];
  r[1] = f[2] * cam->up[0] - f[0] * cam->up[2];
  r[2] = f[0] * cam->up[1] - f[1] * cam->up[0];
  double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(nr > 1e-12)) return fail(c, SPL_EINVAL, "up vector parallel to the view direction");
  for (double &v : r) v /= nr;
  u[0] = r[1] * f[2] - r[2] * f[1];
  u[1] = r[2] * f[0] - r[0] * f[2];
  u[2] = r[0] * f[1] - r[1] * f[0];
  for (int k = 0; k < 3; ++k) {
    pk.e[k] = cam->eye[k];
    pk.r[k] = r[k];
    pk.u[k] = u[k];
    pk.f[k] = f[k];
  }
  pk.F = 0.5 * cam->height / std::tan(0.5 * cam->fov_y_deg * M_PI / 180.0);
  pk.cx = 0.5 * cam->width;
  pk.cy = 0.5 * cam->height;
  pk.z_near = cam->z_near;
  return SPL_OK;
}

spl_status check_params(spl_ctx *c, const spl_params *p, bool need_looks) {
  if (!p) return fail(c, SPL_EINVAL, "params is NULL");
  if (p->mode < SPL_ADD_RAW || p->mode > SPL_SORTED)
    return fail(c, SPL_EINVAL, "unknown mode %d", p->mode);
  if (!(p->nu > 0.0) || !std::isfinite(p->nu)) return fail(c, SPL_EINVAL, "nu must be > 0");
  if (p->tile != 0 && p->tile != 16 && p->tile != 32)
    return fail(c, SPL_EINVAL, "tile must be 0, 16 or 32 (got %d)", p->tile);
  if (p->bin_rule != 0 && p->bin_rule != 1) return fail(c, SPL_EINVAL, "bin_rule must be 0 or 1");
  if (!std::isfinite(p->large_cut)) return fail(c, SPL_EINVAL, "large_cut must be finite");
  if (p->deterministic != 0 && p->deterministic != 1)
    return fail(c, SPL_EINVAL, "deterministic must be 0 or 1");
  if (!need_looks) return SPL_OK;
  if (!(p->k_sigma >= 0.0) || !std::isfinite(p->k_sigma))
    return fail(c, SPL_EINVAL, "k_sigma must be finite and >= 0");
  if (!(p->sigma_min > 0.0) || !std::isfinite(p->sigma_min))
    return fail(c, SPL_EINVAL, "sigma_min must be > 0");
  if (p->n_species < 1 || p->n_species > SPL_MAX_SPECIES)
    return fail(c, SPL_EINVAL, "n_species %d outside 1..%d", p->n_species, SPL_MAX_SPECIES);
  for (int k = 0; k < p->n_species; ++k) {
    const spl_look &l = p->looks[k];
    if (l.vector_colour != 0 && l.vector_colour != 1)
      return fail(c, SPL_EINVAL, "species %d: vector_colour must be 0 or 1", k);
    if (!std::isfinite(l.brightness)) return fail(c, SPL_EINVAL, "species %d: brightness", k);
    if (l.vector_colour) continue;  // the palette fields are not read
    if (!l.rgb) return fail(c, SPL_EINVAL, "palette of species %d is NULL", k);
    if (l.n_entries < 1 || l.n_entries > 4096)
      return fail(c, SPL_EINVAL, "palette of species %d has %d entries", k, l.n_entries);
    if (!std::isfinite(l.lo) || !std::isfinite(l.hi) || !(l.hi >= l.lo))
      return fail(c, SPL_EINVAL, "species %d: need finite lo <= hi", k);
  }
  return SPL_OK;
}

spl_status check_particles(spl_ctx *c, const spl_particles *p, int mode) {
  if (!p) return fail(c, SPL_EINVAL, "particles is NULL");
  if (p->n < 0 || p->n >= (int64_t)0xffffffffll)
    return fail(c, SPL_EINVAL, "particle count %lld outside 0..2^32-2", (long long)p->n);
  if (p->n == 0) return SPL_OK;
  if (!p->x || !p->y || !p->z || !p->h || !p->intensity || !p->scalar)
    return fail(c, SPL_EINVAL, "a required particle array is NULL");
  if (p->attr_dtype < SPL_F32 || p->attr_dtype > SPL_F16)
    return fail(c, SPL_EINVAL, "unknown attr_dtype %d", p->attr_dtype);
  if (!(p->h_scale > 0.0f) || !std::isfinite(p->h_scale) || !(p->i_scale > 0.0f) ||
      !std::isfinite(p->i_scale) || !(p->s_scale > 0.0f) || !std::isfinite(p->s_scale))
    return fail(c, SPL_EINVAL, "h_scale, i_scale and s_scale must be finite and > 0");
  if (mode == SPL_SORTED && !p->absorption)
    return fail(c, SPL_EINVAL, "sorted mode needs absorption");
  if (p->rgb && (!(p->c_scale > 0.0f) || !std::isfinite(p->c_scale)))
    return fail(c, SPL_EINVAL, "c_scale must be finite and > 0");
  return SPL_OK;
}

// A species coloured from the vector field needs the particles' rgb array.
spl_status check_colour(spl_ctx *c, const spl_particles *p, const spl_params *prm) {
  if (p->n == 0) return SPL_OK;
  for (int k = 0; k < prm->n_species; ++k)
    if (prm->looks[k].vector_colour && !p->rgb)
      return fail(c, SPL_EINVAL, "species %d colours from the vector field but rgb is NULL", k);
  return SPL_OK;
}

void fill_proj(ProjK &pk, const spl_particles *p, const spl_params *prm) {
  pk.k_sigma = prm->k_sigma;
  pk.sigma_min = prm->sigma_min;
  pk.nu = prm->nu;
  pk.mode = prm->mode;
  pk.n_species = prm->n_species;
  for (int k = 0; k < SPL_MAX_SPECIES; ++k) {
    LookK &L = pk.looks[k];
    if (k < prm->n_species) {
      const spl_look &l = prm->looks[k];
      L.rgb = l.rgb;
      L.M = l.n_entries;
      L.log10 = l.log10_scalar ? 1 : 0;
      L.vec = l.vector_colour ? 1 : 0;
      L.beta = (float)l.brightness;
      L.lo = (float)l.lo;
      L.inv_range = (l.hi > l.lo) ? (float)(1.0 / (l.hi - l.lo)) : 0.0f;
    } else {
      L = pk.looks[0];
    }
  }
  pk.x = p->x;
  pk.y = p->y;
  pk.z = p->z;
  pk.h = p->h;
  pk.inten = p->intensity;
  pk.scal = p->scalar;
  pk.dtype = p->attr_dtype;
  pk.h_scale = p->h_scale;
  pk.i_scale = p->i_scale;
  pk.s_scale = p->s_scale;
  pk.species = p->species;
  pk.absorb = p->absorption;
  pk.rgb = p->rgb;
  pk.c_scale = p->rgb ? p->c_scale : 1.0f;
  pk.n = p->n;
}

void fill_tiles(TileK &tk, int W, int H, int tile, double nu, double cut, int bin_rule) {
  tk.W = W;
  tk.H = H;
  tk.tile = tile;
  tk.ntx = (W + tile - 1) / tile;
  tk.nty = (H + tile - 1) / tile;
  tk.n_tiles = tk.ntx * tk.nty;
  tk.ctile = kLargeTile;
  const bool large = std::isfinite(cut);
  tk.nctx = large ? (W + kLargeTile - 1) / kLargeTile : 0;
  tk.ncty = large ? (H + kLargeTile - 1) / kLargeTile : 0;
  tk.n_ctiles = tk.nctx * tk.ncty;
  tk.nu = (float)nu;
  tk.large_cut = large ? (float)cut : __builtin_inff();
  tk.bin_rule = bin_rule;
}

// Tile size and large cut for a view: explicit parameters win, then the
// autotuner's cached choice, then the defaults.
// FNV-1a digest of a camera pose (position, look-at, up, field of view,
// near plane): the autotuner's choice depends on the radii the pose projects.
uint64_t pose_digest(const spl_camera *cam) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void *p, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  mix(cam->eye, sizeof(cam->eye));
  mix(cam->lookat, sizeof(cam->lookat));
  mix(cam->up, sizeof(cam->up));
  mix(&cam->fov_y_deg, sizeof(double));
  mix(&cam->z_near, sizeof(double));
  return h;
}

// Tile size and large cut for a view: explicit parameters win, then the
// autotuner's choice for this pose, then its latest choice for the image
// size, then the defaults.
// Lists drawn in list order: depth-sorted, or additive in index order.
bool ordered(const spl_params *prm) {
  return prm->mode == SPL_SORTED || prm->deterministic != 0;
}

// The mode a tuned choice is kept under (the additive modes in index order
// run other kernels than the unordered ones).
int tune_mode(const spl_params *prm) {
  return prm->mode + (prm->mode != SPL_SORTED && prm->deterministic ? 8 : 0);
}

void choose(spl_ctx *c, int64_t n, const spl_camera *cam, const spl_params *prm, int &tile,
            double &cut) {
  tile = prm->tile;
  cut = prm->large_cut;
  const int W = cam->width, H = cam->height;
  const std::pair<int, double> *t = nullptr;
  auto it = c->tune.find(std::make_tuple(n, W, H, tune_mode(prm), pose_digest(cam)));
  if (it != c->tune.end()) {
    t = &it->second;
  } else {
    auto ia = c->tune_any.find(std::make_tuple(n, W, H, tune_mode(prm)));
    if (ia != c->tune_any.end()) t = &ia->second;
  }
  if (tile == 0) tile = t ? t->first : kDefaultTile;
  if (ordered(prm) || cut < 0.0)
    cut = INFINITY;
  else if (cut == 0.0)
    cut = t ? t->second : kDefaultCut;
}

struct Frame {
  int64_t n;
  const float *rec, *rec2;  // rec2 only in sorted mode
  TileK tk;
  int mode, normalise;
  float *out;
  double in_bytes_per_particle;  // bytes the first stage reads per particle
  double out_bytes_per_active;   // bytes it writes per active particle
  bool counted;                  // the first stage already produced the tile counts
  TimedFrame *tf;                // NULL unless timing
  bool flux_check = false;       // expected flux of the records (additive modes)
  bool clear = true;             // zero the image first (else add into it)
  bool finish = true;            // final map, FP64 reductions, normalisation
  bool ordered = false;          // lists sorted on the index, drawn by the composite walk
};

// ---- stage timers ---------------------------------------------------------

hipEvent_t take_event(spl_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  // the stage timers only measure time (no data is read through them), so
  // their events skip the system-scope fence each recording would otherwise
  // wait for
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

bool begin_timed(spl_ctx *c, TimedFrame &tf) {
  for (int k = 0; k <= SPL_N_STAGES; ++k) {
    tf.ev[k] = take_event(c);
    if (!tf.ev[k]) return false;
  }
  for (double &b : tf.bytes) b = 0.0;
  tf.frames = 1;
  return true;
}

void mark(TimedFrame *tf, int k, hipStream_t s) {
  if (tf) (void)hipEventRecord(tf->ev[k], s);  // timing is best effort
}

// Accumulates every pending frame whose last event has completed (all of
// them when wait is true) and returns their events to the pool.
void resolve_timing(spl_ctx *c, bool wait) {
  std::vector<TimedFrame> keep;
  for (TimedFrame &tf : c->pending) {
    hipError_t q = wait ? hipEventSynchronize(tf.ev[SPL_N_STAGES]) : hipEventQuery(tf.ev[SPL_N_STAGES]);
    if (q != hipSuccess) {
      (void)hipGetLastError();
      keep.push_back(tf);
      continue;
    }
    for (int k = 0; k < SPL_N_STAGES; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, tf.ev[k], tf.ev[k + 1]) == hipSuccess) c->acc_ms[k] += ms;
      (void)hipGetLastError();
      c->acc_bytes[k] += tf.bytes[k];
    }
    c->acc_frames += tf.frames;
    for (hipEvent_t e : tf.ev) c->event_pool.push_back(e);
  }
  c->pending.swap(keep);
}

// Reads `bytes` of device memory at src back into page-locked host memory
// (dst_mapped: its device-side address; fine-grained, as h_flag) and waits
// until they are there: the read-back kernel writes them, then, after a
// system-scope fence, this call's sequence number into h_flag, which the
// host watches (a stream synchronisation would add its own wake-up latency
// while the device waits for the host's next launches).  After kSpinMicros
// without the number the host blocks on the stream instead (a long frame, or
// a failed launch whose error the synchronisation then reports).
constexpr int kSpinMicros = 20000;

spl_status readback_wait(spl_ctx *c, const void *src, void *dst_mapped, size_t bytes,
                         hipStream_t s) {
  const uint32_t seq = ++c->rb_seq;
  HIPTRY(c, launch_readback(src, dst_mapped, bytes, s, c->m_flag, seq));
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    if (__atomic_load_n(c->h_flag, __ATOMIC_ACQUIRE) == seq) return SPL_OK;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kSpinMicros)) break;
    __builtin_ia32_pause();
  }
  HIPTRY(c, hipStreamSynchronize(s));
  if (__atomic_load_n(c->h_flag, __ATOMIC_ACQUIRE) != seq)
    return fail(c, SPL_EDEVICE, "read-back of %zu bytes did not arrive", bytes);
  return SPL_OK;
}

// The end of a frame: the absorption = emission map (additive J before it),
// FP64 flux and maximum per channel, optional division by the maximum.
spl_status finish_image(spl_ctx *c, float *img, int64_t npx, int mode, int normalise,
                        hipStream_t s) {
  const int fb = (int)std::min<int64_t>(kFinBlocks, (npx + kBlock - 1) / kBlock);
  HIPTRY(c, launch_finalise(img, npx, mode == SPL_ADD_AEQE, (double *)c->fin.p, fb, s));
  HIPTRY(c, launch_reduce_stats((const double *)c->fin.p, fb, (double *)c->stats.p, s));
  if (normalise) HIPTRY(c, launch_normalise(img, npx, (const double *)c->stats.p, s));
  return SPL_OK;
}

// Everything after the per-particle spans exist (ws span, totals n_active /
// n_large already accumulated, counts zeroed).
spl_status render_lists(spl_ctx *c, const Frame &f, spl_stats *st, hipStream_t s) {
  const TileK &tk = f.tk;
  const int nb = tk.n_tiles + tk.n_ctiles;
  const bool sorted = f.mode == SPL_SORTED;
  // sorted mode (64-bit depth keys), and the additive modes in the stable
  // order (the 32-bit index lists sorted on the index)
  const bool ordered = sorted || f.ordered;
  const int64_t npx = (int64_t)tk.W * tk.H;
  uint32_t *counts = (uint32_t *)c->counts.p, *offsets = (uint32_t *)c->offsets.p,
           *cursor = (uint32_t *)c->cursor.p, *item_off = (uint32_t *)c->item_off.p;
  Totals *tot = (Totals *)c->totals.p;
  const uint2 *span = (const uint2 *)c->span.p;
  TimedFrame *tf = f.tf;

  // unit masks for binning in windows (one word per kUnitParticles)
  TRY(ensure(c, c->umask, (size_t)(f.n / kUnitParticles + 1) * 4));
  uint32_t *umask = (uint32_t *)c->umask.p;
  if (!f.counted) HIPTRY(c, launch_count(span, f.rec, f.n, tk, counts, umask, s));
  mark(tf, 2, s);
  const int chunk[3] = {kChunkSplat, ordered ? kSortChunk : 0, ordered ? kMergeOut : 0};
  const int cchunk[3] = {kChunkLarge, 0, 0};
  const int minc[3] = {1, 1, kSortChunk + 1};
  HIPTRY(c, launch_scan(counts, nb, tk.n_tiles, offsets, cursor, chunk, cchunk, minc, item_off, tot, s));
  mark(tf, 3, s);
  TRY(readback_wait(c, tot, c->m_tot, sizeof(Totals), s));
  if (c->timing) resolve_timing(c, false);
  const Totals T = *c->h_tot;
  if (T.n_pairs >= 0xffffffffull)
    return fail(c, SPL_EUNSUPPORTED, "%llu tile-list entries exceed 2^32", T.n_pairs);
  for (int k = 0; k < 3; ++k)
    if (T.n_items[k] > 0x7fffffffull)
      return fail(c, SPL_EUNSUPPORTED, "too many work items (%llu)", T.n_items[k]);

  // depth order: 64-bit (depth bits, index) keys in two buffers; the stable
  // order: the 32-bit index lists and a second buffer for the merges
  if (sorted) {
    TRY(ensure(c, c->keysA, T.n_pairs * 8));
    TRY(ensure(c, c->keysB, T.n_pairs * 8));
  } else {
    TRY(ensure(c, c->pairs, T.n_pairs * 4));
    if (ordered) TRY(ensure(c, c->keysB, T.n_pairs * 4));
  }
  for (int k = 0; k < 3; ++k) {
    if (chunk[k] == 0) continue;
    TRY(ensure(c, c->items[k], T.n_items[k] * sizeof(Item)));
    if (T.n_items[k])
      HIPTRY(c, launch_build_items(counts, offsets, nb, tk.n_tiles, chunk[k], cchunk[k], minc[k],
                                   item_off + k * (nb + 1), (Item *)c->items[k].p, s));
  }
  unsigned long long *keysA = (unsigned long long *)c->keysA.p;
  unsigned long long *keysB = (unsigned long long *)c->keysB.p;
  mark(tf, 4, s);
  HIPTRY(c, launch_scatter(span, f.rec, f.rec2, f.n, tk, cursor, (uint32_t *)c->pairs.p,
                           sorted ? keysA : nullptr, umask, s));
  mark(tf, 5, s);
  const Item *items0 = (const Item *)c->items[0].p;
  int passes = 0;
  if (!ordered) {
    mark(tf, 6, s);
    if (f.clear) HIPTRY(c, launch_fill_f32(f.out, 0.0f, 3 * npx, s));
    const int nfi = (int)T.n_fine_items[0];
    const int nci = (int)(T.n_items[0] - T.n_fine_items[0]);
    HIPTRY(c, launch_splat_large(items0 + nfi, nci, (const uint32_t *)c->pairs.p, f.rec, counts,
                                 kChunkLarge, tk, f.out, s));
    mark(tf, 7, s);
    HIPTRY(c, launch_splat_add(tk.tile, items0, nfi, (const uint32_t *)c->pairs.p, f.rec, counts,
                               kChunkSplat, tk, f.out, s));
    mark(tf, 8, s);
  } else {
    uint32_t *idxA = (uint32_t *)c->pairs.p, *idxB = (uint32_t *)c->keysB.p;
    const Item *it1 = (const Item *)c->items[1].p, *it2 = (const Item *)c->items[2].p;
    if (sorted)
      HIPTRY(c, launch_sort_chunks(keysA, it1, (int)T.n_items[1], s));
    else
      HIPTRY(c, launch_sort_chunks(idxA, it1, (int)T.n_items[1], s));
    for (int64_t L = kSortChunk; L < (int64_t)T.max_count; L *= 2) {
      if (sorted)
        HIPTRY(c, launch_merge_pass(passes % 2 ? keysB : keysA, passes % 2 ? keysA : keysB, it2,
                                    (int)T.n_items[2], offsets, counts, (int)L, s));
      else
        HIPTRY(c, launch_merge_pass(passes % 2 ? idxB : idxA, passes % 2 ? idxA : idxB, it2,
                                    (int)T.n_items[2], offsets, counts, (int)L, s));
      ++passes;
    }
    mark(tf, 6, s);
    if (f.clear) HIPTRY(c, launch_fill_f32(f.out, 0.0f, 3 * npx, s));
    mark(tf, 7, s);
    const int ni = (int)T.n_items[0];
    TRY(ensure(c, c->partial, (size_t)ni * tk.tile * tk.tile * 16));
    HIPTRY(c, launch_composite(tk.tile, items0, ni, sorted ? (const void *)keysA : idxA,
                               sorted ? (const void *)keysB : idxB, (uint32_t)kSortChunk, f.rec, f.rec2, counts, kChunkSplat, tk,
                               f.out, (float *)c->partial.p, s));
    HIPTRY(c, launch_composite_merge(tk.tile, sorted, items0, ni, counts, kChunkSplat, tk,
                                     (const float *)c->partial.p, f.out, s));
    mark(tf, 8, s);
  }
  if (f.finish) TRY(finish_image(c, f.out, npx, f.mode, f.normalise, s));
  if (f.flux_check)
    HIPTRY(c, launch_expected_flux(f.rec, span, f.n, tk.W, tk.H, tk.nu, (double *)c->fin.p,
                                   kFinBlocks, (double *)c->stats.p + 10, s));
  mark(tf, 9, s);
  if (tf) {
    // algorithmic bytes: every array a stage must touch, once
    const double n = (double)f.n, act = (double)T.n_active, pairs = (double)T.n_pairs;
    const double fine = (double)T.n_fine_pairs, large = pairs - fine;
    const double t2 = (double)tk.tile * tk.tile;
    double *B = tf->bytes;
    B[0] = n * f.in_bytes_per_particle + act * f.out_bytes_per_active + n * 8.0;
    B[1] = f.counted ? 0.0 : n * 8.0 + 4.0 * nb;
    B[2] = 4.0 * nb * 3.0;
    B[3] = 16.0 * (double)(T.n_items[0] + T.n_items[1] + T.n_items[2]);
    B[4] = n * 8.0 + pairs * (sorted ? 8.0 : 4.0);
    // chunk sort: every key read and written once; each merge pass: the
    // keys of the merged lists
    const double kb = sorted ? 16.0 : 8.0;
    B[5] = ordered ? pairs * kb + (double)T.n_merge_keys * kb : 0.0;
    if (!ordered) {
      B[6] = 12.0 * npx + large * 36.0 +
             24.0 * std::min((double)npx, (double)T.n_coarse_nonempty * kLargeTile * kLargeTile);
      B[7] = fine * 36.0 + 24.0 * std::min((double)npx, (double)T.n_fine_nonempty * t2);
    } else {
      B[6] = 12.0 * npx;
      B[7] = pairs * (sorted ? 48.0 : 36.0) +
             12.0 * std::min((double)npx, (double)T.n_fine_nonempty * t2);
    }
    B[8] = (f.mode == SPL_ADD_AEQE ? 24.0 : 12.0) * npx + (f.normalise ? 24.0 * npx : 0.0);
    c->pending.push_back(*tf);
  }
  if (st) {
    if (f.finish || f.flux_check) {
      HIPTRY(c, launch_readback(c->stats.p, c->m_stats, kStatWords * sizeof(double), s));
      HIPTRY(c, hipStreamSynchronize(s));
    }
    st->n_active = (int64_t)T.n_active;
    st->n_large = (int64_t)T.n_large;
    st->n_pairs = (int64_t)T.n_fine_pairs;
    st->n_large_pairs = (int64_t)(T.n_pairs - T.n_fine_pairs);
    st->n_items = (int64_t)T.n_items[0];
    for (int q = 0; q < 3; ++q) {
      st->flux[q] = c->h_stats[q];
      st->max[q] = c->h_stats[3 + q];
      st->raw_flux[q] = sorted ? NAN : c->h_stats[7 + q];
      st->expected_flux[q] = f.flux_check ? c->h_stats[10 + q] : NAN;
    }
    st->tile = tk.tile;
    st->large_cut = std::isfinite(tk.large_cut) ? (double)tk.large_cut : -1.0;
  }
  return SPL_OK;
}

// Runs render_lists with a timed frame when timing is on; on failure the
// frame's events go back to the pool.
spl_status render_timed(spl_ctx *c, Frame &f, TimedFrame *tf, spl_stats *st, hipStream_t s) {
  f.tf = tf;
  spl_status rc = render_lists(c, f, st, s);
  if (rc != SPL_OK && tf)
    for (hipEvent_t e : tf->ev) c->event_pool.push_back(e);
  return rc;
}

spl_status prepare_common(spl_ctx *c, int64_t n, const TileK &tk, hipStream_t s) {
  const int nb = tk.n_tiles + tk.n_ctiles;
  TRY(ensure(c, c->span, (size_t)n * 8));
  TRY(ensure(c, c->counts, (size_t)nb * 4));
  TRY(ensure(c, c->offsets, (size_t)(nb + 1) * 4));
  TRY(ensure(c, c->cursor, (size_t)nb * 4));
  TRY(ensure(c, c->item_off, (size_t)3 * (nb + 1) * 4));
  TRY(ensure(c, c->totals, sizeof(Totals)));
  TRY(ensure(c, c->fin, (size_t)kFinBlocks * kStatPartials * 8));
  TRY(ensure(c, c->stats, kStatWords * 8));
  HIPTRY(c, launch_fill_u32((uint32_t *)c->counts.p, 0u, nb, s));
  HIPTRY(c, launch_fill_u32((uint32_t *)c->totals.p, 0u, sizeof(Totals) / 4, s));
  return SPL_OK;
}

spl_status render_one(spl_ctx *c, const spl_particles *p, const spl_camera *cam,
                      const spl_params *prm, float *out, spl_stats *st, hipStream_t s,
                      bool clear = true, bool finish = true) {
  ProjK pk;
  TRY(check_params(c, prm, true));
  TRY(check_particles(c, p, prm->mode));
  TRY(check_colour(c, p, prm));
  TRY(camera_frame(c, cam, pk));
  if (!out) return fail(c, SPL_EINVAL, "output image is NULL");
  fill_proj(pk, p, prm);
  int tile;
  double cut;
  choose(c, p->n, cam, prm, tile, cut);
  TileK tk;
  fill_tiles(tk, cam->width, cam->height, tile, prm->nu, cut, prm->bin_rule);
  const bool sorted = prm->mode == SPL_SORTED;
  TRY(ensure(c, c->rec, (size_t)p->n * 32));
  if (sorted) TRY(ensure(c, c->rec2, (size_t)p->n * 8));
  TRY(prepare_common(c, p->n, tk, s));
  TimedFrame tfr;
  TimedFrame *tf = (c->timing && begin_timed(c, tfr)) ? &tfr : nullptr;
  mark(tf, 0, s);
  HIPTRY(c, launch_project(pk, tk, (float *)c->rec.p, sorted ? (float *)c->rec2.p : nullptr,
                           (uint2 *)c->span.p, 0, (Totals *)c->totals.p, s,
                           (uint32_t *)c->counts.p));
  mark(tf, 1, s);
  const double attr = p->attr_dtype == SPL_F32 ? 4.0 : 2.0;
  Frame f{p->n, (const float *)c->rec.p, sorted ? (const float *)c->rec2.p : nullptr, tk,
          prm->mode, prm->normalise, out,
          12.0 + 3.0 * attr + (p->species ? 1.0 : 0.0) + (sorted ? 4.0 : 0.0),
          32.0 + (sorted ? 8.0 : 0.0), project_counts(tk), nullptr};
  f.clear = clear;
  f.finish = finish;
  f.flux_check = prm->flux_check != 0 && !sorted;
  f.ordered = ordered(prm);
  return render_timed(c, f, tf, st, s);
}


constexpr int kMaxBatchViews = 255;

spl_status ensure_host(spl_ctx *c, int views) {
  if (c->h_cap >= views) return SPL_OK;
  if (c->h_btot) (void)hipHostFree(c->h_btot);
  if (c->h_views) (void)hipHostFree(c->h_views);
  if (c->h_ctr) (void)hipHostFree(c->h_ctr);
  if (c->h_bstats) (void)hipHostFree(c->h_bstats);
  c->h_btot = nullptr;
  c->h_views = nullptr;
  c->h_ctr = nullptr;
  c->h_bstats = nullptr;
  c->h_cap = 0;
  if (watched_host_alloc((void **)&c->h_btot, sizeof(Totals) * views) != hipSuccess ||
      hipHostMalloc((void **)&c->h_views, sizeof(ViewK) * views, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->h_ctr, 2 * sizeof(uint32_t) * views, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->h_bstats, kStatWords * sizeof(double) * views,
                    hipHostMallocDefault) != hipSuccess)
    return fail(c, SPL_ENOMEM, "pinned host allocation failed");
  if (hipHostGetDevicePointer(&c->m_btot, c->h_btot, 0) != hipSuccess ||
      hipHostGetDevicePointer(&c->m_bstats, c->h_bstats, 0) != hipSuccess)
    return fail(c, SPL_EDEVICE, "device address of pinned host memory unavailable");
  c->h_cap = views;
  return SPL_OK;
}

// One sub-batch of additive views [0, nv): every view's projection, counts
// and scan are launched back to back, one host synchronisation reads all list
// sizes, then the lists of all views are built and splatted by one persistent
// launch (plus one for large particles) and every image is finalised.
spl_status render_views(spl_ctx *c, const spl_particles *p, int nv, const ProjK *pk,
                        const TileK *tk, const spl_params *const *prm, float *const *outs,
                        spl_stats *const *st, hipStream_t s) {
  const int64_t n = p->n;
  int bins = 0;
  for (int v = 0; v < nv; ++v) bins = std::max(bins, tk[v].n_tiles + tk[v].n_ctiles);
  const size_t bstride = (size_t)bins + 1;
  TRY(ensure_host(c, nv));
  TRY(ensure(c, c->b_rec, (size_t)nv * n * 32));
  TRY(ensure(c, c->b_span, (size_t)nv * n * 8));
  TRY(ensure(c, c->b_counts, nv * bstride * 4));
  TRY(ensure(c, c->b_offsets, nv * bstride * 4));
  TRY(ensure(c, c->b_cursor, nv * bstride * 4));
  TRY(ensure(c, c->b_itemoff, (size_t)nv * 3 * bstride * 4));
  TRY(ensure(c, c->b_totals, (size_t)nv * sizeof(Totals)));
  TRY(ensure(c, c->b_views, (size_t)nv * sizeof(ViewK)));
  TRY(ensure(c, c->b_ctr, 4 * sizeof(uint32_t)));
  TRY(ensure(c, c->b_fin, (size_t)nv * kFinBlocks * kStatPartials * 8));
  TRY(ensure(c, c->b_stats, (size_t)nv * kStatWords * 8));
  const size_t mstride = (size_t)(n / kUnitParticles + 1);
  TRY(ensure(c, c->b_umask, (size_t)nv * mstride * 4));
  uint32_t *umask = (uint32_t *)c->b_umask.p;
  float *rec = (float *)c->b_rec.p;
  uint2 *span = (uint2 *)c->b_span.p;
  uint32_t *counts = (uint32_t *)c->b_counts.p, *offsets = (uint32_t *)c->b_offsets.p;
  uint32_t *cursor = (uint32_t *)c->b_cursor.p, *itemoff = (uint32_t *)c->b_itemoff.p;
  Totals *tot = (Totals *)c->b_totals.p;
  const int chunk[3] = {kChunkSplat, kChunkViews, 0}, cchunk[3] = {kChunkLarge, kChunkLarge, 0};
  const int minc[3] = {1, 1, 1};
  // stage timers cover the whole batch (launches without a captured graph):
  // 0 projection, counts and scans of all views, 3 host gap, 4 items,
  // scatter and image clears, 7 both persistent splat launches, 8 finalise
  TimedFrame tfr;
  TimedFrame *tf = (c->timing && !c->graphs && begin_timed(c, tfr)) ? &tfr : nullptr;
  mark(tf, 0, s);
  // the totals and counts of all views cleared at once, every view
  // projected (and counted), then all views' scans in one launch
  HIPTRY(c, launch_fill_u32((uint32_t *)tot, 0u, (int64_t)nv * sizeof(Totals) / 4, s));
  HIPTRY(c, launch_fill_u32(counts, 0u, (int64_t)nv * bstride, s));
  std::vector<int> nbv(nv), nfv(nv);
  for (int v = 0; v < nv; ++v) {
    nbv[v] = tk[v].n_tiles + tk[v].n_ctiles;
    nfv[v] = tk[v].n_tiles;
  }
  for (int v = 0; v < nv;) {
    // two views per pass where both count in the projection: each particle's
    // attributes are then read once for the pair
    if (v + 1 < nv && project_pair_ok(pk[v], tk[v], pk[v + 1], tk[v + 1])) {
      float *const rp[2] = {rec + (size_t)v * n * 8, rec + (size_t)(v + 1) * n * 8};
      uint2 *const sp[2] = {span + (size_t)v * n, span + (size_t)(v + 1) * n};
      Totals *const tp[2] = {tot + v, tot + v + 1};
      uint32_t *const cp[2] = {counts + v * bstride, counts + (v + 1) * bstride};
      HIPTRY(c, launch_project_pair(pk + v, tk + v, rp, sp, tp, cp, s));
      v += 2;
      continue;
    }
    float *rv = rec + (size_t)v * n * 8;
    uint2 *sv = span + (size_t)v * n;
    HIPTRY(c, launch_project(pk[v], tk[v], rv, nullptr, sv, 0, tot + v, s, counts + v * bstride));
    if (!project_counts(tk[v]))
      HIPTRY(c, launch_count(sv, rv, n, tk[v], counts + v * bstride, umask + v * mstride, s));
    ++v;
  }
  HIPTRY(c, launch_scan_views(counts, nv, nbv.data(), nfv.data(), bstride, offsets, cursor, chunk,
                              cchunk, minc, itemoff, tot, s));
  mark(tf, 1, s);
  mark(tf, 2, s);
  mark(tf, 3, s);
  TRY(readback_wait(c, tot, c->m_btot, sizeof(Totals) * nv, s));
  // item length: the long items when there are enough of them for every
  // resident workgroup of the persistent splat
  int ks = 0;
  {
    uint64_t long_items = 0;
    for (int v = 0; v < nv; ++v) long_items += c->h_btot[v].n_fine_items[1];
    const uint64_t slots = (uint64_t)splat_views_resident(tk[0].tile, c->n_cu);
    if (long_items >= (uint64_t)kViewsItemsPerSlot * slots) ks = 1;
  }
  const int ichunk = ks ? kChunkViews : kChunkSplat;
  // views are split into groups whose lists fit 32-bit offsets; the groups
  // run one after another on the stream and reuse the list buffers
  std::vector<int> g0s;
  std::vector<uint64_t> pb(nv), fb(nv), cb(nv), gfine, gcoarse;
  uint64_t max_p = 0, max_f = 0, max_c = 0;
  {
    uint64_t p_run = 0, f_run = 0, c_run = 0;
    for (int v = 0; v < nv; ++v) {
      const Totals &T = c->h_btot[v];
      const uint64_t fi = T.n_fine_items[ks], ci = T.n_items[ks] - T.n_fine_items[ks];
      if (T.n_pairs >= 0xffffffffull || fi > 0x7fffffffull || ci > 0x7fffffffull)
        return fail(c, SPL_EUNSUPPORTED, "view %d: lists too long (%llu entries)", v,
                    (unsigned long long)T.n_pairs);
      if (g0s.empty() || p_run + T.n_pairs > c->group_pairs || f_run + fi > 0x7fffffffull ||
          c_run + ci > 0x7fffffffull) {
        g0s.push_back(v);
        gfine.push_back(0);
        gcoarse.push_back(0);
        p_run = f_run = c_run = 0;
      }
      pb[v] = p_run;
      fb[v] = f_run;
      cb[v] = c_run;
      p_run += T.n_pairs;
      f_run += fi;
      c_run += ci;
      gfine.back() = f_run;
      gcoarse.back() = c_run;
      max_p = std::max(max_p, p_run);
      max_f = std::max(max_f, f_run);
      max_c = std::max(max_c, c_run);
    }
  }
  const int ng = (int)g0s.size();
  g0s.push_back(nv);
  TRY(ensure(c, c->b_pairs, max_p * 4));
  TRY(ensure(c, c->b_itf, max_f * sizeof(Item)));
  TRY(ensure(c, c->b_itc, max_c * sizeof(Item)));
  TRY(ensure(c, c->b_ctr, (size_t)ng * 4 * sizeof(uint32_t)));
  uint32_t *pairs = (uint32_t *)c->b_pairs.p;
  Item *itf = (Item *)c->b_itf.p, *itc = (Item *)c->b_itc.p;
  for (int v = 0; v < nv; ++v) {
    ViewK &vk = c->h_views[v];
    vk.tk = tk[v];
    vk.counts = counts + v * bstride;
    vk.pairs = pairs + pb[v];
    vk.rec = reinterpret_cast<const float4 *>(rec + (size_t)v * n * 8);
    vk.img = outs[v];
  }
  for (int g = 0; g < ng; ++g) {
    c->h_ctr[2 * g] = (uint32_t)gfine[g];
    c->h_ctr[2 * g + 1] = (uint32_t)gcoarse[g];
  }
  // everything after the synchronisation depends only on the list sizes just
  // read; it is enqueued as one unit, directly or as a captured graph
  if (ng != 1 && tf) {  // timers only for a single persistent launch
    for (hipEvent_t e : tf->ev) c->event_pool.push_back(e);
    tf = nullptr;
  }
  auto post = [&](hipStream_t q) -> spl_status {
    mark(tf, 4, q);
    for (int g = 0; g < ng; ++g) {
      const int v0 = g0s[g], v1 = g0s[g + 1];
      // the work items of the group's views, one launch per kMaxLaunchViews
      // views (views without items write none)
      for (int a = v0; a < v1; a += kMaxLaunchViews) {
        const int b = std::min(v1, a + kMaxLaunchViews);
        ItemViews iv;
        for (int v = a; v < b; ++v) {
          iv.nb[v - a] = nbv[v];
          iv.n_fine[v - a] = nfv[v];
          iv.fine[v - a] = (uint32_t)fb[v];
          iv.coarse[v - a] = (uint32_t)cb[v];
          iv.coarse_shift[v - a] = (uint32_t)c->h_btot[v].n_fine_items[ks];
          iv.view[v - a] = (uint32_t)(v - v0);
        }
        HIPTRY(c, launch_build_items_views(counts + a * bstride, offsets + a * bstride, bstride,
                                           ichunk, kChunkLarge, 1, itemoff + 3 * a * bstride, ks,
                                           itf, itc, iv, b - a, q));
      }
      for (int v = v0; v < v1; ++v)
        HIPTRY(c, launch_scatter(span + (size_t)v * n, rec + (size_t)v * n * 8, nullptr, n,
                                 tk[v], cursor + v * bstride, pairs + pb[v], nullptr,
                                 umask + v * mstride, q));
      for (int a = v0; a < v1; a += kMaxLaunchViews) {
        const int b = std::min(v1, a + kMaxLaunchViews);
        ImgViews iv;
        for (int v = a; v < b; ++v) {
          iv.img[v - a] = outs[v];
          iv.n_px[v - a] = (int64_t)tk[v].W * tk[v].H;
        }
        HIPTRY(c, launch_clear_views(iv, b - a, q));
      }
      ViewK *dviews = (ViewK *)c->b_views.p + v0;
      uint32_t *ctr = (uint32_t *)c->b_ctr.p + 4 * g;
      HIPTRY(c, hipMemcpyAsync(dviews, c->h_views + v0, sizeof(ViewK) * (v1 - v0),
                               hipMemcpyHostToDevice, q));
      HIPTRY(c, hipMemcpyAsync(ctr, c->h_ctr + 2 * g, 2 * sizeof(uint32_t), hipMemcpyHostToDevice,
                               q));
      HIPTRY(c, launch_fill_u32(ctr + 2, 0u, 2, q));
      mark(tf, 5, q);
      mark(tf, 6, q);
      mark(tf, 7, q);
      HIPTRY(c, launch_splat_views(tk[0].tile, dviews, itf, ctr, ctr + 2, itc, ctr + 1, ctr + 3,
                                   ichunk, kChunkLarge, c->n_cu, gcoarse[g] > 0, q));
      mark(tf, 8, q);
      double *fin = (double *)c->b_fin.p, *stats = (double *)c->b_stats.p;
      // the final map and FP64 reductions of the group's views, one launch
      // each per kMaxLaunchViews views
      const size_t pstride = (size_t)kFinBlocks * kStatPartials;
      for (int a = v0; a < v1; a += kMaxLaunchViews) {
        const int b = std::min(v1, a + kMaxLaunchViews);
        ImgViews iv;
        for (int v = a; v < b; ++v) {
          const int64_t npx = (int64_t)tk[v].W * tk[v].H;
          iv.img[v - a] = outs[v];
          iv.n_px[v - a] = npx;
          iv.blocks[v - a] = (int)std::min<int64_t>(kFinBlocks, (npx + kBlock - 1) / kBlock);
          iv.aeqe[v - a] = prm[v]->mode == SPL_ADD_AEQE;
        }
        HIPTRY(c, launch_finalise_views(iv, b - a, fin + a * pstride, pstride, q));
        HIPTRY(c, launch_reduce_stats_views(fin + a * pstride, pstride, iv, b - a,
                                            stats + (size_t)kStatWords * a, kStatWords, q));
      }
      for (int v = v0; v < v1; ++v) {
        const int64_t npx = (int64_t)tk[v].W * tk[v].H;
        if (prm[v]->normalise)
          HIPTRY(c, launch_normalise(outs[v], npx, stats + kStatWords * v, q));
        if (prm[v]->flux_check)
          HIPTRY(c, launch_expected_flux(rec + (size_t)v * n * 8, span + (size_t)v * n, n,
                                         tk[v].W, tk[v].H, tk[v].nu,
                                         fin + (size_t)v * kFinBlocks * kStatPartials, kFinBlocks,
                                         stats + kStatWords * v + 10, q));
      }
    }
    mark(tf, 9, q);
    return SPL_OK;
  };
  if (!c->graphs) {
    TRY(post(s));
  } else {
    // capture on the context's own stream (the null stream cannot be
    // captured), then replay on the caller's stream; the executable graph is
    // kept and updated in place while the launch topology stays the same
    if (!c->cap_stream) HIPTRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPTRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const spl_status cs = post(c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(c->cap_stream, &graph);
    if (cs != SPL_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cs;
    }
    if (ce != hipSuccess) return fail(c, SPL_EDEVICE, "graph capture failed: %s", hipGetErrorString(ce));
    hipError_t e = hipSuccess;
    if (c->gexec) {
      hipGraphNode_t bad = nullptr;
      hipGraphExecUpdateResult res;
      if (hipGraphExecUpdate(c->gexec, graph, &bad, &res) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
      }
    }
    if (!c->gexec) e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(c->gexec, s);
    if (e != hipSuccess) return fail(c, SPL_EDEVICE, "graph launch failed: %s", hipGetErrorString(e));
  }
  if (tf) {
    // algorithmic bytes of the batch, summed over its views (same figures as
    // the single-view frame)
    const double attr = p->attr_dtype == SPL_F32 ? 4.0 : 2.0;
    const double in_pp = 12.0 + 3.0 * attr + (p->species ? 1.0 : 0.0);
    double *B = tf->bytes;
    for (int v = 0; v < nv; ++v) {
      const Totals &T = c->h_btot[v];
      const double act = (double)T.n_active, pairs = (double)T.n_pairs;
      const double fine = (double)T.n_fine_pairs, large = pairs - fine;
      const double npx = (double)tk[v].W * tk[v].H, t2 = (double)tk[v].tile * tk[v].tile;
      const double nbv = (double)(tk[v].n_tiles + tk[v].n_ctiles);
      B[0] += (double)n * in_pp + act * 32.0 + (double)n * 8.0 +
              (project_counts(tk[v]) ? 0.0 : (double)n * 8.0 + 4.0 * nbv) + 12.0 * nbv;
      B[4] += 16.0 * (double)T.n_items[ks] + (double)n * 8.0 + pairs * 4.0 + 12.0 * npx;
      B[7] += fine * 36.0 + 24.0 * std::min(npx, (double)T.n_fine_nonempty * t2) + large * 36.0 +
              24.0 * std::min(npx, (double)T.n_coarse_nonempty * kLargeTile * kLargeTile);
      B[8] += 24.0 * npx;
    }
    tf->frames = nv;
    c->pending.push_back(*tf);
  }
  double *stats = (double *)c->b_stats.p;
  bool any_stats = false;
  for (int v = 0; v < nv; ++v) any_stats = any_stats || st[v];
  if (any_stats) {
    HIPTRY(c, launch_readback(stats, c->m_bstats, kStatWords * sizeof(double) * nv, s));
    HIPTRY(c, hipStreamSynchronize(s));
    for (int v = 0; v < nv; ++v) {
      if (!st[v]) continue;
      const Totals &T = c->h_btot[v];
      st[v]->n_active = (int64_t)T.n_active;
      st[v]->n_large = (int64_t)T.n_large;
      st[v]->n_pairs = (int64_t)T.n_fine_pairs;
      st[v]->n_large_pairs = (int64_t)(T.n_pairs - T.n_fine_pairs);
      st[v]->n_items = (int64_t)T.n_items[ks];
      for (int q = 0; q < 3; ++q) {
        const double *hs = c->h_bstats + kStatWords * v;
        st[v]->flux[q] = hs[q];
        st[v]->max[q] = hs[3 + q];
        st[v]->raw_flux[q] = hs[7 + q];
        st[v]->expected_flux[q] = prm[v]->flux_check ? hs[10 + q] : NAN;
      }
      st[v]->tile = tk[v].tile;
      st[v]->large_cut = std::isfinite(tk[v].large_cut) ? (double)tk[v].large_cut : -1.0;
    }
  }
  return SPL_OK;
}

spl_status render_batch(spl_ctx *c, const spl_particles *p, int nv, const spl_camera *cams,
                        const spl_params *prms, float *const *outs, spl_stats *st,
                        hipStream_t s) {
  TRY(check_particles(c, p, SPL_ADD_RAW));
  std::vector<ProjK> pk;
  std::vector<TileK> tk;
  std::vector<const spl_params *> pv;
  std::vector<float *> ov;
  std::vector<spl_stats *> sv;
  // every view is validated before any work is enqueued
  bool any_sorted = false;
  for (int v = 0; v < nv; ++v) {
    ProjK k;
    TRY(check_params(c, &prms[v], true));
    TRY(check_colour(c, p, &prms[v]));
    TRY(camera_frame(c, &cams[v], k));
    if (!outs[v]) return fail(c, SPL_EINVAL, "output image %d is NULL", v);
    any_sorted = any_sorted || prms[v].mode == SPL_SORTED;
  }
  if (any_sorted) TRY(check_particles(c, p, SPL_SORTED));
  for (int v = 0; v < nv; ++v) {
    // views drawn in list order (depth-sorted, or additive in index order)
    // take the single-view path
    if (ordered(&prms[v])) {
      TRY(render_one(c, p, &cams[v], &prms[v], outs[v], st ? &st[v] : nullptr, s));
      continue;
    }
    ProjK k;
    camera_frame(c, &cams[v], k);
    fill_proj(k, p, &prms[v]);
    int tile;
    double cut;
    choose(c, p->n, &cams[v], &prms[v], tile, cut);
    TileK t;
    fill_tiles(t, cams[v].width, cams[v].height, tile, prms[v].nu, cut, prms[v].bin_rule);
    pk.push_back(k);
    tk.push_back(t);
    pv.push_back(&prms[v]);
    ov.push_back(outs[v]);
    sv.push_back(st ? &st[v] : nullptr);
  }
  const int na = (int)pk.size();
  if (na == 0) return SPL_OK;
  // one persistent launch serves one tile size: views are taken tile size by
  // tile size (each keeps the tile it would get on its own), in call order
  // within a size; the images are independent, so the order is free
  std::vector<int> order(na);
  for (int v = 0; v < na; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return tk[a].tile < tk[b].tile; });
  std::vector<ProjK> pk2(na);
  std::vector<TileK> tk2(na);
  std::vector<const spl_params *> pv2(na);
  std::vector<float *> ov2(na);
  std::vector<spl_stats *> sv2(na);
  for (int i = 0; i < na; ++i) {
    const int v = order[i];
    pk2[i] = pk[v];
    tk2[i] = tk[v];
    pv2[i] = pv[v];
    ov2[i] = ov[v];
    sv2[i] = sv[v];
  }
  // views per launch: what the memory budget allows (records, spans and about
  // two list entries per particle, per view)
  const int64_t per_view = p->n * (32 + 8 + 8) + ((int64_t)4 << 20);
  const int per = (int)std::max<int64_t>(
      1, std::min<int64_t>(kMaxBatchViews, c->budget / std::max<int64_t>(per_view, 1)));
  for (int v0 = 0; v0 < na;) {
    int m = 1;
    while (m < per && v0 + m < na && tk2[v0 + m].tile == tk2[v0].tile) ++m;
    TRY(render_views(c, p, m, &pk2[v0], &tk2[v0], &pv2[v0], &ov2[v0], &sv2[v0], s));
    v0 += m;
  }
  return SPL_OK;
}

// ---- resident data sets ----------------------------------------------------

size_t attr_bytes(int dtype) { return dtype == SPL_F32 ? 4 : 2; }
size_t round256(size_t v) { return (v + 255) & ~(size_t)255; }

hipError_t copy_in(void *dst, const void *src, size_t bytes, int on_device, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        s);
}

// One attribute array (count values) into the stored type; returns the scale
// of the stored values in *scale_out.
spl_status convert_attr(spl_ctx *c, const void *src, int sdtype, float sscale, int64_t count,
                        int on_device, void *stage, void *dst, int store, float *scale_out,
                        hipStream_t s) {
  const void *from = src;
  if (!on_device) {
    HIPTRY(c, copy_in(stage, src, (size_t)count * attr_bytes(sdtype), 0, s));
    from = stage;
  }
  double scale = 1.0;
  if (store == SPL_F16) {
    // the power of two that puts the largest finite magnitude in [2^10, 2^11)
    uint32_t *bits = (uint32_t *)c->minmax.p;
    HIPTRY(c, launch_fill_u32(bits, 0u, 1, s));
    HIPTRY(c, launch_absmax(from, sdtype, sscale, count, bits, s));
    uint32_t hb = 0;
    HIPTRY(c, hipMemcpyAsync(&hb, bits, 4, hipMemcpyDeviceToHost, s));
    HIPTRY(c, hipStreamSynchronize(s));
    float m;
    std::memcpy(&m, &hb, 4);
    if (m > 0.0f) scale = std::ldexp(1.0, (int)std::floor(std::log2((double)m / 1024.0)));
  }
  HIPTRY(c, launch_convert(from, sdtype, sscale, dst, store, (float)(1.0 / scale), count, s));
  *scale_out = (float)scale;
  return SPL_OK;
}

spl_status dataset_upload(spl_ctx *c, const spl_particles *src, int on_device, int store,
                          spl_dataset **out, hipStream_t s) {
  if (!out) return fail(c, SPL_EINVAL, "out is NULL");
  TRY(check_particles(c, src, SPL_ADD_RAW));
  if (store < SPL_F32 || store > SPL_F16)
    return fail(c, SPL_EINVAL, "unknown store_dtype %d", store);
  const int64_t n = src->n;
  const size_t sa = attr_bytes(store), ssrc = attr_bytes(src->attr_dtype);
  // layout of the one allocation
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round256(bytes);
    return o;
  };
  const size_t ox = take(4 * n), oy = take(4 * n), oz = take(4 * n);
  const size_t oh = take(sa * n), oi = take(sa * n), os = take(sa * n);
  const size_t osp = src->species ? take(n) : 0;
  const size_t oab = src->absorption ? take(4 * n) : 0;
  const size_t orgb = src->rgb ? take(3 * sa * n) : 0;
  spl_dataset *ds = new (std::nothrow) spl_dataset();
  if (!ds) return fail(c, SPL_ENOMEM, "host allocation failed");
  if (hipMalloc(&ds->mem, off ? off : 256) != hipSuccess) {
    (void)hipGetLastError();
    delete ds;
    return fail(c, SPL_ENOMEM, "device allocation of %zu bytes for the data set failed", off);
  }
  ds->bytes = off;
  ds->device = c->device;
  char *m = (char *)ds->mem;
  void *stage = nullptr;
  spl_status rc = SPL_OK;
  auto cleanup = [&](spl_status r) {
    if (stage) (void)hipFree(stage);
    if (r != SPL_OK) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(ds->mem);
      delete ds;
    }
    return r;
  };
  if (n > 0) {
    if (!on_device &&
        hipMalloc(&stage, (size_t)n * ssrc * (src->rgb ? 3 : 1)) != hipSuccess) {
      (void)hipGetLastError();
      stage = nullptr;
      return cleanup(fail(c, SPL_ENOMEM, "device staging allocation failed"));
    }
    if ((rc = ensure(c, c->minmax, 4 * SPL_MAX_SPECIES * 8)) != SPL_OK) return cleanup(rc);
    const hipError_t e0 = copy_in(m + ox, src->x, 4 * n, on_device, s);
    const hipError_t e1 = e0 == hipSuccess ? copy_in(m + oy, src->y, 4 * n, on_device, s) : e0;
    const hipError_t e2 = e1 == hipSuccess ? copy_in(m + oz, src->z, 4 * n, on_device, s) : e1;
    const hipError_t e3 = (e2 == hipSuccess && src->species) ? copy_in(m + osp, src->species, n, on_device, s) : e2;
    const hipError_t e4 = (e3 == hipSuccess && src->absorption)
                              ? copy_in(m + oab, src->absorption, 4 * n, on_device, s)
                              : e3;
    if (e4 != hipSuccess)
      return cleanup(fail(c, SPL_EDEVICE, "data set copy failed: %s", hipGetErrorString(e4)));
    float sc = 1.0f;
    if ((rc = convert_attr(c, src->h, src->attr_dtype, src->h_scale, n, on_device, stage, m + oh,
                           store, &sc, s)) != SPL_OK)
      return cleanup(rc);
    ds->view.h_scale = sc;
    if ((rc = convert_attr(c, src->intensity, src->attr_dtype, src->i_scale, n, on_device, stage,
                           m + oi, store, &sc, s)) != SPL_OK)
      return cleanup(rc);
    ds->view.i_scale = sc;
    if ((rc = convert_attr(c, src->scalar, src->attr_dtype, src->s_scale, n, on_device, stage,
                           m + os, store, &sc, s)) != SPL_OK)
      return cleanup(rc);
    ds->view.s_scale = sc;
    ds->view.c_scale = 1.0f;
    if (src->rgb) {
      if ((rc = convert_attr(c, src->rgb, src->attr_dtype, src->c_scale, 3 * n, on_device, stage,
                             m + orgb, store, &sc, s)) != SPL_OK)
        return cleanup(rc);
      ds->view.c_scale = sc;
    }
    if (hipStreamSynchronize(s) != hipSuccess)
      return cleanup(fail(c, SPL_EDEVICE, "data set upload failed"));
  } else {
    ds->view.h_scale = ds->view.i_scale = ds->view.s_scale = ds->view.c_scale = 1.0f;
  }
  spl_particles &v = ds->view;
  v.n = n;
  v.x = (const float *)(m + ox);
  v.y = (const float *)(m + oy);
  v.z = (const float *)(m + oz);
  v.h = m + oh;
  v.intensity = m + oi;
  v.scalar = m + os;
  v.attr_dtype = store;
  v.species = src->species ? (const uint8_t *)(m + osp) : nullptr;
  v.absorption = src->absorption ? (const float *)(m + oab) : nullptr;
  v.rgb = src->rgb ? (const void *)(m + orgb) : nullptr;
  *out = ds;
  return cleanup(SPL_OK);
}

spl_status check_dataset(spl_ctx *c, const spl_dataset *ds) {
  if (!ds) return fail(c, SPL_EINVAL, "data set is NULL");
  if (ds->device != c->device)
    return fail(c, SPL_EINVAL, "data set lives on device %d, the context on %d", ds->device,
                c->device);
  return SPL_OK;
}

// A frame into a host image: rendered into the context's device image, then
// copied back (Sect. 3.1: the image goes back to the host at the end).
spl_status render_out(spl_ctx *c, const spl_particles *p, const spl_camera *cam,
                      const spl_params *prm, float *out, int out_on_device, spl_stats *st,
                      hipStream_t s) {
  if (out_on_device) return render_one(c, p, cam, prm, out, st, s);
  if (!out) return fail(c, SPL_EINVAL, "output image is NULL");
  if (!cam || cam->width < 1 || cam->height < 1 || cam->width > 32768 || cam->height > 32768)
    return fail(c, SPL_EINVAL, "bad camera or image size");
  const size_t bytes = (size_t)cam->width * cam->height * 12;
  TRY(ensure(c, c->himg, bytes));
  TRY(render_one(c, p, cam, prm, (float *)c->himg.p, st, s));
  HIPTRY(c, hipMemcpyAsync(out, c->himg.p, bytes, hipMemcpyDeviceToHost, s));
  HIPTRY(c, hipStreamSynchronize(s));
  return SPL_OK;
}

spl_status render_batch_out(spl_ctx *c, const spl_particles *p, int nv, const spl_camera *cams,
                            const spl_params *prms, float *const *outs, int out_on_device,
                            spl_stats *st, hipStream_t s) {
  if (out_on_device) return render_batch(c, p, nv, cams, prms, outs, st, s);
  size_t total = 0;
  for (int v = 0; v < nv; ++v) {
    if (!outs[v]) return fail(c, SPL_EINVAL, "output image %d is NULL", v);
    if (cams[v].width < 1 || cams[v].height < 1 || cams[v].width > 32768 ||
        cams[v].height > 32768)
      return fail(c, SPL_EINVAL, "view %d: image size %dx%d outside 1..32768", v, cams[v].width,
                  cams[v].height);
    total += round256((size_t)cams[v].width * cams[v].height * 12);
  }
  TRY(ensure(c, c->himg, total));
  std::vector<float *> dev(nv);
  size_t off = 0;
  for (int v = 0; v < nv; ++v) {
    dev[v] = (float *)((char *)c->himg.p + off);
    off += round256((size_t)cams[v].width * cams[v].height * 12);
  }
  TRY(render_batch(c, p, nv, cams, prms, dev.data(), st, s));
  for (int v = 0; v < nv; ++v)
    HIPTRY(c, hipMemcpyAsync(outs[v], dev[v], (size_t)cams[v].width * cams[v].height * 12,
                             hipMemcpyDeviceToHost, s));
  HIPTRY(c, hipStreamSynchronize(s));
  return SPL_OK;
}

// ---- out-of-core rendering --------------------------------------------------

// Chunk k of the host arrays into device buffer b (one allocation per buffer:
// positions, attributes, species, colour vectors), on the copy stream, after
// the render that last read the buffer.
spl_status stream_copy(spl_ctx *c, const spl_particles *hp, int64_t chunk, int64_t k,
                       spl_particles *views) {
  const int b = (int)(k & 1);
  const int64_t first = k * chunk, m = std::min<int64_t>(chunk, hp->n - first);
  const size_t sa = attr_bytes(hp->attr_dtype);
  char *base = (char *)c->chunk[b].p;
  size_t off = 0;
  auto take = [&](size_t per) {
    char *p = base + off;
    off += round256(per * (size_t)chunk);
    return p;
  };
  spl_particles &v = views[b];
  v = *hp;
  v.n = m;
  float *x = (float *)take(4), *y = (float *)take(4), *z = (float *)take(4);
  void *h = take(sa), *in = take(sa), *sc = take(sa);
  uint8_t *sp = hp->species ? (uint8_t *)take(1) : nullptr;
  void *rgb = hp->rgb ? take(3 * sa) : nullptr;
  hipStream_t q = c->copy_stream;
  if (k >= 2) HIPTRY(c, hipStreamWaitEvent(q, c->ev_done[b], 0));
  HIPTRY(c, copy_in(x, hp->x + first, 4 * m, 0, q));
  HIPTRY(c, copy_in(y, hp->y + first, 4 * m, 0, q));
  HIPTRY(c, copy_in(z, hp->z + first, 4 * m, 0, q));
  HIPTRY(c, copy_in(h, (const char *)hp->h + sa * first, sa * m, 0, q));
  HIPTRY(c, copy_in(in, (const char *)hp->intensity + sa * first, sa * m, 0, q));
  HIPTRY(c, copy_in(sc, (const char *)hp->scalar + sa * first, sa * m, 0, q));
  if (sp) HIPTRY(c, copy_in(sp, hp->species + first, m, 0, q));
  if (rgb) HIPTRY(c, copy_in(rgb, (const char *)hp->rgb + 3 * sa * first, 3 * sa * m, 0, q));
  HIPTRY(c, hipEventRecord(c->ev_copied[b], q));
  v.x = x;
  v.y = y;
  v.z = z;
  v.h = h;
  v.intensity = in;
  v.scalar = sc;
  v.species = sp;
  v.rgb = rgb;
  v.absorption = nullptr;
  return SPL_OK;
}

spl_status render_stream(spl_ctx *c, const spl_particles *hp, int64_t chunk,
                         const spl_camera *cam, const spl_params *prm, float *img,
                         spl_stats *st, hipStream_t s) {
  TRY(check_params(c, prm, true));
  if (prm->mode == SPL_SORTED)
    return fail(c, SPL_EUNSUPPORTED, "out-of-core rendering is additive only (depth order "
                                     "spans chunks)");
  TRY(check_particles(c, hp, prm->mode));
  TRY(check_colour(c, hp, prm));
  ProjK pk;
  TRY(camera_frame(c, cam, pk));
  if (!img) return fail(c, SPL_EINVAL, "output image is NULL");
  if (chunk < 1) return fail(c, SPL_EINVAL, "chunk must be >= 1");
  chunk = std::min<int64_t>(chunk, std::max<int64_t>(hp->n, 1));
  if (!c->copy_stream) HIPTRY(c, hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
  for (int b = 0; b < 2; ++b) {
    if (!c->ev_copied[b])
      HIPTRY(c, hipEventCreateWithFlags(&c->ev_copied[b], hipEventDisableTiming));
    if (!c->ev_done[b]) HIPTRY(c, hipEventCreateWithFlags(&c->ev_done[b], hipEventDisableTiming));
  }
  const size_t sa = attr_bytes(hp->attr_dtype);
  const size_t per = round256(4 * chunk) * 3 + round256(sa * chunk) * 3 +
                     (hp->species ? round256(chunk) : 0) + (hp->rgb ? round256(3 * sa * chunk) : 0);
  TRY(ensure(c, c->chunk[0], per));
  TRY(ensure(c, c->chunk[1], per));
  TRY(ensure(c, c->fin, (size_t)kFinBlocks * kStatPartials * 8));  // an empty set renders no
  TRY(ensure(c, c->stats, kStatWords * 8));                          // chunk but is finished
  // the chunk frames: the transfer sum J added into the image, no map
  spl_params q = *prm;
  q.mode = SPL_ADD_RAW;
  q.normalise = 0;
  // the tile size and cut the whole set would get
  int tile;
  double cut;
  choose(c, hp->n, cam, prm, tile, cut);
  q.tile = tile;
  q.large_cut = std::isfinite(cut) ? cut : -1.0;
  const int64_t npx = (int64_t)cam->width * cam->height;
  const int64_t nchunks = (hp->n + chunk - 1) / chunk;
  HIPTRY(c, launch_fill_f32(img, 0.0f, 3 * npx, s));
  const bool timing = c->timing;
  c->timing = false;  // per-chunk stage timers would count chunks as frames
  spl_particles views[2];
  spl_stats acc{};
  spl_status rc = SPL_OK;
  double expected[3] = {0.0, 0.0, 0.0};
  // the copy stream may start once the image clear and earlier work on the
  // caller's stream are ordered before it
  hipEvent_t start = c->ev_done[1];
  HIPTRY(c, hipEventRecord(start, s));
  HIPTRY(c, hipStreamWaitEvent(c->copy_stream, start, 0));
  if (nchunks > 0) rc = stream_copy(c, hp, chunk, 0, views);
  for (int64_t k = 0; k < nchunks && rc == SPL_OK; ++k) {
    const int b = (int)(k & 1);
    if (k + 1 < nchunks && (rc = stream_copy(c, hp, chunk, k + 1, views)) != SPL_OK) break;
    if (hipStreamWaitEvent(s, c->ev_copied[b], 0) != hipSuccess) {
      rc = fail(c, SPL_EDEVICE, "stream wait failed");
      break;
    }
    spl_stats cs{};
    rc = render_one(c, &views[b], cam, &q, img, &cs, s, false, false);
    if (rc != SPL_OK) break;
    if (hipEventRecord(c->ev_done[b], s) != hipSuccess) {
      rc = fail(c, SPL_EDEVICE, "event record failed");
      break;
    }
    acc.n_active += cs.n_active;
    acc.n_large += cs.n_large;
    acc.n_pairs += cs.n_pairs;
    acc.n_large_pairs += cs.n_large_pairs;
    acc.n_items += cs.n_items;
    for (int ch = 0; ch < 3; ++ch) expected[ch] += cs.expected_flux[ch];
  }
  c->timing = timing;
  if (rc != SPL_OK) {
    (void)hipStreamSynchronize(c->copy_stream);
    return rc;
  }
  HIPTRY(c, hipStreamSynchronize(c->copy_stream));
  // the map, the FP64 reductions and the normalisation, once, on the sum
  TRY(finish_image(c, img, npx, prm->mode, prm->normalise, s));
  if (st) {
    HIPTRY(c, launch_readback(c->stats.p, c->m_stats, kStatWords * sizeof(double), s));
    HIPTRY(c, hipStreamSynchronize(s));
    *st = acc;
    for (int ch = 0; ch < 3; ++ch) {
      st->flux[ch] = c->h_stats[ch];
      st->max[ch] = c->h_stats[3 + ch];
      st->raw_flux[ch] = c->h_stats[7 + ch];
      st->expected_flux[ch] = prm->flux_check ? expected[ch] : NAN;
    }
    st->tile = tile;
    st->large_cut = std::isfinite(cut) ? cut : -1.0;
  } else {
    HIPTRY(c, hipStreamSynchronize(s));
  }
  return SPL_OK;
}

}  // namespace

extern "C" {

spl_status spl_create(int device, spl_ctx **out) {
  if (!out) return SPL_EINVAL;
  *out = nullptr;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || nd <= 0) {
    (void)hipGetLastError();
    return SPL_EDEVICE;
  }
  if (device < 0 || device >= nd) return SPL_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return SPL_EDEVICE;
  // the device address of this device's `scratch` (once per device, with
  // the device current)
  void *scratch_ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < kMaxDevices && g_scratch[device]) {
      scratch_ptr = g_scratch[device];
    } else {
      const hipError_t e = hipGetSymbolAddress(&scratch_ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !scratch_ptr) {
        (void)hipGetLastError();
        return SPL_EDEVICE;
      }
      if (device < kMaxDevices) g_scratch[device] = scratch_ptr;
    }
  }
  spl_ctx *c = new (std::nothrow) spl_ctx();
  if (!c) return SPL_ENOMEM;
  c->device = device;
  c->scratch = scratch_ptr;
  c->err.reserve(512);  // error messages then need no allocation
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->n_cu = ncu;
  if (watched_host_alloc((void **)&c->h_tot, sizeof(Totals)) != hipSuccess ||
      hipHostMalloc((void **)&c->h_stats, kStatWords * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      watched_host_alloc((void **)&c->h_flag, 64) != hipSuccess) {
    if (c->h_tot) (void)hipHostFree(c->h_tot);
    if (c->h_stats) (void)hipHostFree(c->h_stats);
    delete c;
    return SPL_ENOMEM;
  }
  *c->h_flag = 0;
  if (hipHostGetDevicePointer(&c->m_tot, c->h_tot, 0) != hipSuccess ||
      hipHostGetDevicePointer(&c->m_stats, c->h_stats, 0) != hipSuccess ||
      hipHostGetDevicePointer(&c->m_flag, c->h_flag, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(c->h_tot);
    (void)hipHostFree(c->h_stats);
    (void)hipHostFree(c->h_flag);
    delete c;
    return SPL_EDEVICE;
  }
  *out = c;
  return SPL_OK;
}

// Every workspace buffer of the context, for release.
#define SPL_WORKSPACE_BUFFERS(c)                                                            \
  {&c->rec, &c->rec2, &c->span, &c->counts, &c->offsets, &c->cursor, &c->item_off,          \
   &c->items[0], &c->items[1], &c->items[2], &c->pairs, &c->keysA, &c->keysB, &c->partial,  \
   &c->fin, &c->stats, &c->totals, &c->minmax, &c->b_rec, &c->b_span, &c->b_counts,          \
   &c->b_offsets, &c->b_cursor, &c->b_itemoff, &c->b_totals, &c->b_pairs, &c->b_itf,        \
   &c->b_itc, &c->b_views, &c->b_ctr, &c->b_fin, &c->b_stats, &c->himg, &c->chunk[0],        \
   &c->chunk[1], &c->umask, &c->b_umask}

spl_status spl_trim(spl_ctx *c) {
  if (!c) return SPL_EINVAL;
  HIPTRY(c, hipSetDevice(c->device));
  HIPTRY(c, hipDeviceSynchronize());  // no frame may still use the buffers
  DevBuf *bufs[] = SPL_WORKSPACE_BUFFERS(c);
  for (DevBuf *b : bufs) {
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->cap = 0;
  }
  c->bytes = 0;
  if (c->gexec) {  // the replayable graph points into the freed buffers
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  return SPL_OK;
}

void spl_destroy(spl_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  DevBuf *bufs[] = SPL_WORKSPACE_BUFFERS(c);
  for (DevBuf *b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (TimedFrame &tf : c->pending)
    for (hipEvent_t e : tf.ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->h_tot) (void)hipHostFree(c->h_tot);
  if (c->h_stats) (void)hipHostFree(c->h_stats);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  if (c->h_btot) (void)hipHostFree(c->h_btot);
  if (c->h_views) (void)hipHostFree(c->h_views);
  if (c->h_ctr) (void)hipHostFree(c->h_ctr);
  if (c->h_bstats) (void)hipHostFree(c->h_bstats);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  for (int b = 0; b < 2; ++b) {
    if (c->ev_copied[b]) (void)hipEventDestroy(c->ev_copied[b]);
    if (c->ev_done[b]) (void)hipEventDestroy(c->ev_done[b]);
  }
  delete c;
}

const char *spl_last_error(const spl_ctx *c) {
  if (!c) return "no context";
  return c->err.c_str();
}

int64_t spl_workspace_bytes(const spl_ctx *c) { return c ? c->bytes : 0; }

spl_status spl_scalar_range(spl_ctx *c, const spl_particles *p, int32_t n_species,
                            int32_t log10_scalar, double *lo, double *hi, void *stream) {
  if (!c) return SPL_EINVAL;
  if (!lo || !hi) return fail(c, SPL_EINVAL, "lo / hi is NULL");
  if (n_species < 1 || n_species > SPL_MAX_SPECIES)
    return fail(c, SPL_EINVAL, "n_species %d outside 1..%d", n_species, SPL_MAX_SPECIES);
  if (!p || p->n < 0) return fail(c, SPL_EINVAL, "bad particle set");
  if (p->n > 0 && !p->scalar) return fail(c, SPL_EINVAL, "scalar array is NULL");
  if (p->attr_dtype < SPL_F32 || p->attr_dtype > SPL_F16)
    return fail(c, SPL_EINVAL, "unknown attr_dtype %d", p->attr_dtype);
  HIPTRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  TRY(ensure(c, c->minmax, 4 * SPL_MAX_SPECIES * 8));
  ProjK pk;
  std::memset(&pk, 0, sizeof(pk));
  pk.scal = p->scalar;
  pk.species = p->species;
  pk.dtype = p->attr_dtype;
  pk.s_scale = (p->s_scale > 0.0f && std::isfinite(p->s_scale)) ? p->s_scale : 1.0f;
  pk.n = p->n;
  HIPTRY(c, launch_scalar_range(pk, n_species, log10_scalar ? 1 : 0, (double *)c->minmax.p, s));
  double h[2 * SPL_MAX_SPECIES];
  HIPTRY(c, hipMemcpyAsync(h, (double *)c->minmax.p + 2 * SPL_MAX_SPECIES,
                           2 * SPL_MAX_SPECIES * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPTRY(c, hipStreamSynchronize(s));
  for (int k = 0; k < n_species; ++k) {
    lo[k] = h[2 * k];
    hi[k] = h[2 * k + 1];
  }
  return SPL_OK;
}

spl_status spl_project(spl_ctx *c, const spl_particles *p, const spl_camera *cam,
                       const spl_params *prm, float *rec, float *rec2, void *stream) {
  if (!c) return SPL_EINVAL;
  ProjK pk;
  TRY(check_params(c, prm, true));
  TRY(check_particles(c, p, prm->mode));
  TRY(check_colour(c, p, prm));
  TRY(camera_frame(c, cam, pk));
  if (p->n > 0 && !rec) return fail(c, SPL_EINVAL, "rec is NULL");
  HIPTRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  fill_proj(pk, p, prm);
  TileK tk;
  fill_tiles(tk, cam->width, cam->height, kDefaultTile, prm->nu, INFINITY, 0);
  TRY(ensure(c, c->span, (size_t)p->n * 8));
  TRY(ensure(c, c->totals, sizeof(Totals)));
  HIPTRY(c, launch_fill_u32((uint32_t *)c->totals.p, 0u, sizeof(Totals) / 4, s));
  HIPTRY(c, launch_project(pk, tk, rec, rec2, (uint2 *)c->span.p, 1, (Totals *)c->totals.p, s));
  return SPL_OK;
}

spl_status spl_bin(spl_ctx *c, int64_t n, const float *rec, const float *rec2, int32_t width,
                   int32_t height, int32_t tile, double nu, int32_t bin_rule, int32_t by_depth,
                   uint32_t *counts, uint32_t *offsets, uint32_t *pairs, int64_t pairs_cap,
                   int64_t *n_pairs, void *stream) {
  if (!c) return SPL_EINVAL;
  if (n < 0 || n >= (int64_t)0xffffffffll) return fail(c, SPL_EINVAL, "bad record count");
  if (n > 0 && !rec) return fail(c, SPL_EINVAL, "rec is NULL");
  if (by_depth < 0 || by_depth > 2) return fail(c, SPL_EINVAL, "by_depth must be 0, 1 or 2");
  if (by_depth == 1 && n > 0 && !rec2) return fail(c, SPL_EINVAL, "by_depth 1 needs rec2");
  if (width < 1 || height < 1 || width > 32768 || height > 32768 || tile < 1)
    return fail(c, SPL_EINVAL, "bad image or tile size");
  if (!(nu > 0.0)) return fail(c, SPL_EINVAL, "nu must be > 0");
  if (bin_rule != 0 && bin_rule != 1) return fail(c, SPL_EINVAL, "bin_rule must be 0 or 1");
  if (!counts || !offsets || !n_pairs) return fail(c, SPL_EINVAL, "output array is NULL");
  TileK tk;
  fill_tiles(tk, width, height, tile, nu, INFINITY, bin_rule);
  if ((int64_t)tk.ntx * tk.nty > (1 << 24)) return fail(c, SPL_EINVAL, "more than 2^24 tiles");
  HIPTRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const int nb = tk.n_tiles;
  TRY(ensure(c, c->span, (size_t)n * 8));
  TRY(ensure(c, c->cursor, (size_t)nb * 4));
  TRY(ensure(c, c->item_off, (size_t)3 * (nb + 1) * 4));
  TRY(ensure(c, c->totals, sizeof(Totals)));
  HIPTRY(c, launch_fill_u32(counts, 0u, nb, s));
  HIPTRY(c, launch_fill_u32((uint32_t *)c->totals.p, 0u, sizeof(Totals) / 4, s));
  Totals *tot = (Totals *)c->totals.p;
  HIPTRY(c, launch_span_from_records(rec, n, tk, (uint2 *)c->span.p, tot, s));
  TRY(ensure(c, c->umask, (size_t)(n / kUnitParticles + 1) * 4));
  uint32_t *umask = (uint32_t *)c->umask.p;
  HIPTRY(c, launch_count((const uint2 *)c->span.p, rec, n, tk, counts, umask, s));
  const int chunk[3] = {0, by_depth ? kSortChunk : 0, by_depth ? kMergeOut : 0};
  const int cchunk[3] = {0, 0, 0};
  const int minc[3] = {1, 1, kSortChunk + 1};
  uint32_t *item_off = (uint32_t *)c->item_off.p;
  HIPTRY(c, launch_scan(counts, nb, nb, offsets, (uint32_t *)c->cursor.p, chunk, cchunk, minc,
                        item_off, tot, s));
  HIPTRY(c, launch_readback(tot, c->m_tot, sizeof(Totals), s));
  HIPTRY(c, hipStreamSynchronize(s));
  const Totals T = *c->h_tot;
  if (T.n_pairs >= 0xffffffffull) return fail(c, SPL_EUNSUPPORTED, "too many list entries");
  *n_pairs = (int64_t)T.n_pairs;
  if (!pairs) return SPL_OK;
  if ((int64_t)T.n_pairs > pairs_cap)
    return fail(c, SPL_ENOMEM, "pairs_cap %lld < %llu entries", (long long)pairs_cap, T.n_pairs);
  if (!by_depth) {
    HIPTRY(c, launch_scatter((const uint2 *)c->span.p, rec, rec2, n, tk, (uint32_t *)c->cursor.p,
                             pairs, nullptr, umask, s));
    HIPTRY(c, hipStreamSynchronize(s));
    return SPL_OK;
  }
  for (int k = 1; k < 3; ++k) {
    TRY(ensure(c, c->items[k], T.n_items[k] * sizeof(Item)));
    if (T.n_items[k])
      HIPTRY(c, launch_build_items(counts, offsets, nb, nb, chunk[k], 0, minc[k],
                                   item_off + k * (nb + 1), (Item *)c->items[k].p, s));
  }
  if (by_depth == 2) {
    // the stable order: the index lists sorted in place (the merge passes'
    // second buffer in the workspace)
    TRY(ensure(c, c->keysB, T.n_pairs * 4));
    uint32_t *B2 = (uint32_t *)c->keysB.p;
    HIPTRY(c, launch_scatter((const uint2 *)c->span.p, rec, nullptr, n, tk,
                             (uint32_t *)c->cursor.p, pairs, nullptr, umask, s));
    HIPTRY(c, launch_sort_chunks(pairs, (const Item *)c->items[1].p, (int)T.n_items[1], s));
    int passes = 0;
    for (int64_t L = kSortChunk; L < (int64_t)T.max_count; L *= 2) {
      HIPTRY(c, launch_merge_pass(passes % 2 ? B2 : pairs, passes % 2 ? pairs : B2,
                                  (const Item *)c->items[2].p, (int)T.n_items[2], offsets, counts,
                                  (int)L, s));
      ++passes;
    }
    if (passes > 0)
      HIPTRY(c, launch_copy_items(B2, pairs, (const Item *)c->items[2].p, (int)T.n_items[2],
                                  counts, (uint32_t)kSortChunk, s));
    HIPTRY(c, hipStreamSynchronize(s));
    return SPL_OK;
  }
  TRY(ensure(c, c->keysA, T.n_pairs * 8));
  TRY(ensure(c, c->keysB, T.n_pairs * 8));
  unsigned long long *A = (unsigned long long *)c->keysA.p, *B = (unsigned long long *)c->keysB.p;
  HIPTRY(c, launch_scatter((const uint2 *)c->span.p, rec, rec2, n, tk, (uint32_t *)c->cursor.p,
                           nullptr, A, umask, s));
  HIPTRY(c, launch_sort_chunks(A, (const Item *)c->items[1].p, (int)T.n_items[1], s));
  int passes = 0;
  for (int64_t L = kSortChunk; L < (int64_t)T.max_count; L *= 2) {
    HIPTRY(c, launch_merge_pass(passes % 2 ? B : A, passes % 2 ? A : B,
                                (const Item *)c->items[2].p, (int)T.n_items[2], offsets, counts,
                                (int)L, s));
    ++passes;
  }
  // lists short enough for one in-LDS sort never leave A; a merged list ends
  // in B after an odd number of its own passes and is copied back
  if (passes > 0)
    HIPTRY(c, launch_copy_items(B, A, (const Item *)c->items[2].p, (int)T.n_items[2], counts,
                                (uint32_t)kSortChunk, s));
  HIPTRY(c, launch_keys_to_pids(A, (int64_t)T.n_pairs, pairs, s));
  HIPTRY(c, hipStreamSynchronize(s));
  return SPL_OK;
}

spl_status spl_render_records(spl_ctx *c, int64_t n, const float *rec, const float *rec2,
                              const spl_camera *cam, const spl_params *prm, float *out,
                              spl_stats *st, void *stream) {
  if (!c) return SPL_EINVAL;
  TRY(check_params(c, prm, false));
  if (!cam || cam->width < 1 || cam->height < 1 || cam->width > 32768 || cam->height > 32768)
    return fail(c, SPL_EINVAL, "bad image size");
  if (n < 0 || n >= (int64_t)0xffffffffll) return fail(c, SPL_EINVAL, "bad record count");
  if (n > 0 && !rec) return fail(c, SPL_EINVAL, "rec is NULL");
  if (prm->mode == SPL_SORTED && n > 0 && !rec2)
    return fail(c, SPL_EINVAL, "sorted mode needs rec2");
  if (!out) return fail(c, SPL_EINVAL, "output image is NULL");
  HIPTRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  int tile;
  double cut;
  choose(c, n, cam, prm, tile, cut);
  TileK tk;
  fill_tiles(tk, cam->width, cam->height, tile, prm->nu, cut, prm->bin_rule);
  TRY(prepare_common(c, n, tk, s));
  TimedFrame tfr;
  TimedFrame *tf = (c->timing && begin_timed(c, tfr)) ? &tfr : nullptr;
  mark(tf, 0, s);
  HIPTRY(c, launch_span_from_records(rec, n, tk, (uint2 *)c->span.p, (Totals *)c->totals.p, s));
  mark(tf, 1, s);
  Frame f{n, rec, prm->mode == SPL_SORTED ? rec2 : nullptr, tk, prm->mode, prm->normalise, out,
          32.0, 0.0, false, nullptr};
  f.ordered = ordered(prm);
  return render_timed(c, f, tf, st, s);
}

spl_status spl_set_timing(spl_ctx *c, int32_t enable) {
  if (!c) return SPL_EINVAL;
  c->timing = enable != 0;
  return SPL_OK;
}

spl_status spl_get_timing(spl_ctx *c, double *ms, double *bytes, int64_t *frames) {
  if (!c) return SPL_EINVAL;
  if (!ms || !bytes || !frames) return fail(c, SPL_EINVAL, "output arrays are NULL");
  HIPTRY(c, hipSetDevice(c->device));
  resolve_timing(c, true);
  for (int k = 0; k < SPL_N_STAGES; ++k) {
    ms[k] = c->acc_ms[k];
    bytes[k] = c->acc_bytes[k];
    c->acc_ms[k] = 0.0;
    c->acc_bytes[k] = 0.0;
  }
  *frames = c->acc_frames;
  c->acc_frames = 0;
  return SPL_OK;
}

spl_status spl_render(spl_ctx *c, const spl_particles *p, const spl_camera *cam,
                      const spl_params *prm, float *out, spl_stats *st, void *stream) {
  if (!c) return SPL_EINVAL;
  HIPTRY(c, hipSetDevice(c->device));
  return render_one(c, p, cam, prm, out, st, (hipStream_t)stream);
}

spl_status spl_render_noalloc(spl_ctx *c, const spl_particles *p, const spl_camera *cam,
                              const spl_params *prm, float *out, spl_stats *st, void *stream) {
  if (!c) return SPL_EINVAL;
  TRY(check_params(c, prm, true));
  TRY(check_particles(c, p, prm->mode));
  TRY(check_colour(c, p, prm));
  if (!c->scratch) return fail(c, SPL_EDEVICE, "scratch address unknown on device %d", c->device);
  HIPTRY(c, hipSetDevice(c->device));
  // the per-particle buffers bound the particle count up front; the lists,
  // whose size the frame learns after its count, are checked when carved
  const bool sorted = prm->mode == SPL_SORTED;
  const size_t per_particle = 32 + 8 + (sorted ? 8 : 0);
  const size_t fixed = (size_t)kFinBlocks * kStatPartials * 8 + kStatWords * 8 +
                       sizeof(Totals) + 4096;
  if (p->n > 0 && (size_t)p->n > (kScratchBytes - fixed) / per_particle)
    return fail(c, SPL_ENOMEM,
                "%lld particles need %zu bytes of per-particle workspace; the %zu-byte scratch "
                "holds at most %zu particles in this mode",
                (long long)p->n, (size_t)p->n * per_particle, kScratchBytes,
                (kScratchBytes - fixed) / per_particle);
  // the frame's buffers come from the scratch: the context's own workspace
  // is set aside and restored afterwards
  Arena a;
  a.base = (char *)c->scratch;
  a.cap = kScratchBytes;
  DevBuf *bufs[] = {&c->rec,      &c->rec2,     &c->span,  &c->counts,  &c->offsets,
                    &c->cursor,   &c->item_off, &c->items[0], &c->items[1], &c->items[2],
                    &c->pairs,    &c->keysA,    &c->keysB, &c->partial, &c->fin,
                    &c->stats,    &c->totals,   &c->umask};
  constexpr int kBufs = (int)(sizeof(bufs) / sizeof(bufs[0]));
  DevBuf saved[kBufs];
  for (int k = 0; k < kBufs; ++k) {
    saved[k] = *bufs[k];
    *bufs[k] = DevBuf();
  }
  const bool timing = c->timing;
  c->timing = false;  // stage timers create events
  c->arena = &a;
  const spl_status rc = render_one(c, p, cam, prm, out, st, (hipStream_t)stream);
  c->arena = nullptr;
  c->timing = timing;
  for (int k = 0; k < kBufs; ++k) *bufs[k] = saved[k];
  return rc;
}

int64_t spl_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

spl_status spl_render_batch(spl_ctx *c, const spl_particles *p, int32_t n_views,
                            const spl_camera *cams, const spl_params *prms, float *const *outs,
                            spl_stats *st, void *stream) {
  if (!c) return SPL_EINVAL;
  if (n_views < 0 || (n_views > 0 && (!cams || !prms || !outs)))
    return fail(c, SPL_EINVAL, "bad view arrays");
  HIPTRY(c, hipSetDevice(c->device));
  if (n_views == 0) return SPL_OK;
  return render_batch(c, p, n_views, cams, prms, outs, st, (hipStream_t)stream);
}

spl_status spl_dataset_upload(spl_ctx *c, const spl_particles *src, int32_t src_on_device,
                              int32_t store_dtype, spl_dataset **out, void *stream) {
  if (!c) return SPL_EINVAL;
  HIPTRY(c, hipSetDevice(c->device));
  return dataset_upload(c, src, src_on_device ? 1 : 0, store_dtype, out, (hipStream_t)stream);
}

void spl_dataset_free(spl_dataset *ds) {
  if (!ds) return;
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  (void)hipSetDevice(ds->device);
  (void)hipDeviceSynchronize();  // no render may still read it
  if (ds->mem) (void)hipFree(ds->mem);
  if (have) (void)hipSetDevice(cur);
  delete ds;
}

spl_status spl_dataset_particles(const spl_dataset *ds, spl_particles *out) {
  if (!ds || !out) return SPL_EINVAL;
  *out = ds->view;
  return SPL_OK;
}

int64_t spl_dataset_bytes(const spl_dataset *ds) { return ds ? (int64_t)ds->bytes : 0; }

spl_status spl_render_dataset(spl_ctx *c, const spl_dataset *ds, const spl_camera *cam,
                              const spl_params *prm, float *out, int32_t out_on_device,
                              spl_stats *st, void *stream) {
  if (!c) return SPL_EINVAL;
  TRY(check_dataset(c, ds));
  HIPTRY(c, hipSetDevice(c->device));
  return render_out(c, &ds->view, cam, prm, out, out_on_device, st, (hipStream_t)stream);
}

spl_status spl_render_batch_dataset(spl_ctx *c, const spl_dataset *ds, int32_t n_views,
                                    const spl_camera *cams, const spl_params *prms,
                                    float *const *outs, int32_t out_on_device, spl_stats *st,
                                    void *stream) {
  if (!c) return SPL_EINVAL;
  TRY(check_dataset(c, ds));
  if (n_views < 0 || (n_views > 0 && (!cams || !prms || !outs)))
    return fail(c, SPL_EINVAL, "bad view arrays");
  HIPTRY(c, hipSetDevice(c->device));
  if (n_views == 0) return SPL_OK;
  return render_batch_out(c, &ds->view, n_views, cams, prms, outs, out_on_device, st,
                          (hipStream_t)stream);
}

spl_status spl_render_stream(spl_ctx *c, const spl_particles *p, int64_t chunk,
                             const spl_camera *cam, const spl_params *prm, float *out,
                             int32_t out_on_device, spl_stats *st, void *stream) {
  if (!c) return SPL_EINVAL;
  HIPTRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (out_on_device) return render_stream(c, p, chunk, cam, prm, out, st, s);
  if (!out) return fail(c, SPL_EINVAL, "output image is NULL");
  if (!cam || cam->width < 1 || cam->height < 1 || cam->width > 32768 || cam->height > 32768)
    return fail(c, SPL_EINVAL, "bad camera or image size");
  const size_t bytes = (size_t)cam->width * cam->height * 12;
  TRY(ensure(c, c->himg, bytes));
  TRY(render_stream(c, p, chunk, cam, prm, (float *)c->himg.p, st, s));
  HIPTRY(c, hipMemcpyAsync(out, c->himg.p, bytes, hipMemcpyDeviceToHost, s));
  HIPTRY(c, hipStreamSynchronize(s));
  return SPL_OK;
}

spl_status spl_host_alloc(size_t bytes, void **out) {
  if (!out) return SPL_EINVAL;
  *out = nullptr;
  if (hipHostMalloc(out, bytes ? bytes : 1, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return SPL_ENOMEM;
  }
  return SPL_OK;
}

void spl_host_free(void *p) {
  if (p) (void)hipHostFree(p);
}

spl_status spl_set_option(spl_ctx *c, int32_t option, int64_t value) {
  if (!c) return SPL_EINVAL;
  switch (option) {
    case SPL_OPT_TIMING:
      c->timing = value != 0;
      return SPL_OK;
    case SPL_OPT_GRAPHS:
      c->graphs = value != 0;
      return SPL_OK;
    case SPL_OPT_BATCH_BYTES:
      if (value <= 0) return fail(c, SPL_EINVAL, "batch budget must be > 0");
      c->budget = value;
      return SPL_OK;
    case SPL_OPT_BATCH_PAIRS:
      if (value < 1 || value > (int64_t)0xfffffffell)
        return fail(c, SPL_EINVAL, "list entries per launch must be in 1..2^32-2");
      c->group_pairs = (uint64_t)value;
      return SPL_OK;
    default:
      return fail(c, SPL_EINVAL, "unknown option %d", option);
  }
}

spl_status spl_autotune(spl_ctx *c, const spl_particles *p, const spl_camera *cam,
                        const spl_params *prm, int32_t *tile_out, double *cut_out, void *stream) {
  if (!c) return SPL_EINVAL;
  if (!tile_out || !cut_out) return fail(c, SPL_EINVAL, "outputs are NULL");
  TRY(check_params(c, prm, true));
  TRY(check_particles(c, p, prm->mode));
  TRY(check_colour(c, p, prm));
  ProjK pk;
  TRY(camera_frame(c, cam, pk));
  HIPTRY(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  float *img = nullptr;
  if (hipMalloc(&img, (size_t)cam->width * cam->height * 12) != hipSuccess)
    return fail(c, SPL_ENOMEM, "autotune image allocation failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(img);
    return fail(c, SPL_EDEVICE, "autotune event creation failed");
  }
  const int tiles[2] = {16, 32};
  const double cuts_add[5] = {16.0, 32.0, 64.0, 128.0, -1.0};
  const double cuts_sorted[1] = {-1.0};
  const double *cuts = ordered(prm) ? cuts_sorted : cuts_add;
  const int ncut = ordered(prm) ? 1 : 5;
  float best = INFINITY;
  int best_tile = kDefaultTile;
  double best_cut = kDefaultCut;
  spl_status rc = SPL_OK;
  for (int ti = 0; ti < 2 && rc == SPL_OK; ++ti)
    for (int ci = 0; ci < ncut && rc == SPL_OK; ++ci) {
      spl_params q = *prm;
      q.tile = tiles[ti];
      q.large_cut = cuts[ci];
      float tmin = INFINITY;
      for (int rep = 0; rep < 3 && rc == SPL_OK; ++rep) {
        hipError_t e = hipEventRecord(e0, s);
        rc = render_one(c, p, cam, &q, img, nullptr, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess && rc == SPL_OK)
          rc = fail(c, SPL_EDEVICE, "autotune timing failed: %s", hipGetErrorString(e));
        if (rep > 0 && ms < tmin) tmin = ms;
      }
      if (tmin < best) {
        best = tmin;
        best_tile = tiles[ti];
        best_cut = cuts[ci] < 0 ? -1.0 : cuts[ci];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(img);
  if (rc != SPL_OK) return rc;
  const std::pair<int, double> choice(best_tile, best_cut < 0 ? INFINITY : best_cut);
  c->tune[std::make_tuple(p->n, cam->width, cam->height, tune_mode(prm), pose_digest(cam))] = choice;
  c->tune_any[std::make_tuple(p->n, cam->width, cam->height, tune_mode(prm))] = choice;
  *tile_out = best_tile;
  *cut_out = best_cut;
  return SPL_OK;
}

}  // extern "C"
