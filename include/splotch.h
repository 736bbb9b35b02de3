/*
 * splotch.h -- C ABI of the MI355X (gfx950) Splotch render library.
 *
 * Method: Dykes, Gheller, Rivi, Krokos, "Splotch: porting and optimizing for
 * the Xeon Phi" (arXiv:1606.04427).  The calls follow the problem statement of
 * Sect. 2.1: particle arrays (positions, radius, scalar fields), camera and
 * look-at positions, colour maps loaded at run time and render parameters go
 * in; a single-precision RGB image comes out.  Sect. 3.1 fixes the render
 * organisation (square tiles, one particle list per tile, each tile's pixels
 * owned by one worker).
 *
 * Conventions shared by every call:
 *  - Device pointers are HIP device memory on the context's device; host
 *    pointers are marked "host".  The caller owns every array it passes in
 *    and every output buffer; the library owns only its context workspace.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *    on it; calls that return host values (counts, statistics, ranges)
 *    synchronise that stream before returning.
 *  - Every call returns an spl_status.  On error nothing is written to
 *    out-parameters and spl_last_error() describes the failure.  No C++
 *    exception crosses the ABI.
 *  - A context is not thread-safe: one host thread per context.
 *  - Images are height x width x 3 float32, row-major, row 0 at the top,
 *    channel-minor.  Pixel (i, j) covers [i, i+1) x [j, j+1).
 */
#ifndef SPLOTCH_H
#define SPLOTCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPL_OK = 0,
  SPL_EINVAL = -1,      /* invalid argument (camera, parameters, sizes) */
  SPL_ENOMEM = -2,      /* device allocation failed */
  SPL_EDEVICE = -3,     /* HIP runtime error (no device, launch failure) */
  SPL_EBUSY = -4,       /* request refused by the memory budget */
  SPL_EUNSUPPORTED = -5 /* valid request the library does not handle */
} spl_status;

typedef enum { SPL_F32 = 0, SPL_BF16 = 1, SPL_F16 = 2 } spl_dtype;

/* Radiative-transfer modes (Sect. 2.1, "radiative transfer equation";
 * Sect. 3.2.2, additive drawing of colour x contribution). */
typedef enum {
  SPL_ADD_RAW = 0,  /* J = sum_p E_p tau_p */
  SPL_ADD_AEQE = 1, /* absorption = emission: I = 1 - exp(-J) */
  SPL_SORTED = 2    /* separate absorption, depth-ordered slab compositing */
} spl_mode;

#define SPL_MAX_SPECIES 8

/* Particles, structure of arrays, device memory (Sect. 2.1: positions,
 * radius, scalar fields; Sect. 4.1: gas and star species). */
typedef struct {
  int64_t n;
  const float *x, *y, *z;    /* world positions, n floats each */
  const void *h;             /* smoothing length, n x attr_dtype */
  const void *intensity;     /* n x attr_dtype */
  const void *scalar;        /* colour scalar, n x attr_dtype */
  int32_t attr_dtype;        /* spl_dtype of h, intensity, scalar */
  float h_scale;             /* smoothing length = h_scale * h (world units) */
  float i_scale;             /* intensity = i_scale * intensity */
  float s_scale;             /* colour scalar = s_scale * scalar; the scales let
                                FP16 storage keep values in range (use 1 for
                                FP32 and BF16) */
  const uint8_t *species;    /* n bytes, or NULL (all species 0) */
  const float *absorption;   /* n floats, SPL_SORTED only, else ignored */
  const void *rgb;           /* colour vector field (Sect. 2.1: colour taken
                                directly from a vector input field), n x 3
                                attr_dtype, row per particle; NULL unless a
                                species colours from it */
  float c_scale;             /* colour vector = c_scale * rgb */
} spl_particles;

/* Camera and look-at positions (Sect. 2.1).  Forward = lookat - eye, right =
 * forward x up, vertical field of view in degrees, (0, 180).  Particles at
 * view depth <= z_near are clipped.  1 <= width, height <= 32768. */
typedef struct {
  double eye[3], lookat[3], up[3];
  double fov_y_deg, z_near;
  int32_t width, height;
} spl_camera;

/* One look per species (Sect. 2.1: colour generated either as a function of
 * a scalar through a colour map loaded at run time, or directly from a
 * vector input field; the scene file varies brightness and palette
 * thresholds).  Palette colouring (vector_colour = 0): rgb is device memory,
 * n_entries x 3 floats, entries evenly spaced over the normalised scalar; the
 * (log10 if log10_scalar) scalar is normalised by [lo, hi], hi >= lo.
 * Vector colouring (vector_colour = 1): the colour is the particle's own
 * rgb vector (spl_particles.rgb, required); palette fields are ignored.
 * Either way the emission is brightness x intensity x colour. */
typedef struct {
  const float *rgb;
  int32_t n_entries;    /* 1 .. 4096 */
  int32_t log10_scalar;
  double brightness;
  double lo, hi;
  int32_t vector_colour;
} spl_look;

typedef struct {
  int32_t mode;       /* spl_mode */
  int32_t n_species;  /* 1 .. SPL_MAX_SPECIES */
  spl_look looks[SPL_MAX_SPECIES];
  double k_sigma;     /* kernel width sigma = sqrt((k_sigma rho)^2 + sigma_min^2) */
  double sigma_min;   /* px, > 0 */
  double nu;          /* truncation radius R = nu sigma, > 0 */
  int32_t tile;       /* tile edge in px: 16 or 32; 0 = library choice */
  int32_t bin_rule;   /* 0 = every tile the pixel box touches; 1 = the paper's
                         0.75 R + sqrt(2) tile/2 distance threshold */
  double large_cut;   /* px: particles with R > large_cut take the large-
                         particle path (additive modes); 0 = library choice,
                         < 0 = never */
  int32_t normalise;  /* 1: divide the image by its maximum value */
  int32_t flux_check; /* additive modes, 1: also compute the expected flux
                         (spl_stats.expected_flux), one more pass over the
                         particles' pixel boxes */
  int32_t deterministic; /* additive modes, 1: the image is the same bit for
                         bit on every run (Sect. 3.1: each tile's pixels are
                         drawn by the one worker that owns them, so nothing
                         races).  Each tile list is put in ascending particle
                         index (the scatter's list, then a sort of each list
                         on the index) and drawn in that order: per pixel the
                         contributions are summed in list order, long lists
                         in chunk order.  The large-particle path is off.
                         Costs about what the depth sort of SPL_SORTED costs.
                         0: sums in an order the device schedule picks
                         (reproducible to rounding).  Ignored in SPL_SORTED,
                         which is always deterministic. */
} spl_params;

/* Per-render statistics; flux and max are FP64 reductions over the final
 * image.  Stage times are filled only when timing is enabled. */
typedef struct {
  int64_t n_active;      /* particles that reach the image */
  int64_t n_large;       /* of which on the large-particle path */
  int64_t n_pairs;       /* (particle, tile) entries in the tile lists */
  int64_t n_large_pairs; /* (particle, large tile) entries */
  int64_t n_items;       /* splat work items */
  double flux[3];        /* sum over pixels, per channel */
  double max[3];         /* maximum pixel value, per channel */
  int32_t tile;          /* tile size used */
  double large_cut;      /* large-particle cut used, px */
  double raw_flux[3];    /* additive modes: sum over pixels of J = sum_p E_p
                            tau_p before the absorption = emission map (FP64) */
  double expected_flux[3]; /* flux_check: sum over particles of E_p kappa_p,
                            kappa_p = the particle's sampled, truncated and
                            clipped kernel summed over its pixels (FP64
                            accumulation); equals raw_flux up to rounding when
                            every contribution reaches the image; NaN
                            otherwise */
} spl_stats;

typedef struct spl_ctx spl_ctx;

typedef struct spl_dataset spl_dataset;

/* Creates a context bound to `device`: one stream-ordered worker with a
 * device workspace that grows on demand and is reused by every later frame
 * (Sect. 3.2.1: allocation on the hot path is a large cost, so buffers are
 * pooled and reused rather than allocated per frame). */
spl_status spl_create(int device, spl_ctx **out);
void spl_destroy(spl_ctx *ctx);
/* Message for the last failed call on this context (never NULL). */
const char *spl_last_error(const spl_ctx *ctx);
/* Device memory currently held by the context workspace, bytes. */
int64_t spl_workspace_bytes(const spl_ctx *ctx);
/* Releases the context workspace (after the device finishes its work); the
 * next frame allocates what it needs again.  For callers that share a device
 * memory budget between several contexts. */
spl_status spl_trim(spl_ctx *ctx);

/* Ranging (Sect. 2.1 preprocessing): per-species min / max of the scalar
 * field, or of log10 of it (values <= 0 skipped), over finite values.  lo, hi:
 * host arrays of n_species doubles; a species without values gets
 * +inf / -inf.  Synchronises. */
spl_status spl_scalar_range(spl_ctx *ctx, const spl_particles *p, int32_t n_species,
                            int32_t log10_scalar, double *lo, double *hi, void *stream);

/* Transform, projection, clipping and colour (Sect. 2.1 rasterisation;
 * Sect. 3.1 transform and colour loops).  Writes, per particle, the record
 * rec[8p..8p+7] = {Xi, Xf, Yi, Yf, sigma, Ar, Ag, Ab}: screen position split in
 * integer part and fraction (X = Xi + Xf), kernel width in px, and emission
 * premultiplied by the kernel amplitude 1/(pi sigma^2).  Clipped particles get
 * an all-zero record (sigma = 0).  rec2 (may be NULL) gets {a/(pi sigma^2),
 * view depth} per particle.  Device arrays of 8n and 2n floats. */
spl_status spl_project(spl_ctx *ctx, const spl_particles *p, const spl_camera *cam,
                       const spl_params *prm, float *rec, float *rec2, void *stream);

/* Tile lists from records (Sect. 3.1; tile-list pseudocode figure): counts
 * (n_tiles), offsets (n_tiles + 1, exclusive scan) and pairs (particle
 * indices grouped by tile).  Within a tile, pairs are in ascending
 * (view-depth bits, index) order when by_depth = 1 (needs rec2), in ascending
 * index when by_depth = 2 (the stable order), and in no specified order when
 * by_depth = 0.  tile: any edge >= 1 px.  Device arrays; *n_pairs
 * (host) gets the total.  SPL_ENOMEM if pairs_cap is too small (counts and
 * offsets are still written).  Synchronises. */
spl_status spl_bin(spl_ctx *ctx, int64_t n, const float *rec, const float *rec2,
                   int32_t width, int32_t height, int32_t tile, double nu,
                   int32_t bin_rule, int32_t by_depth, uint32_t *counts,
                   uint32_t *offsets, uint32_t *pairs, int64_t pairs_cap,
                   int64_t *n_pairs, void *stream);

/* Renders records made by spl_project (same camera size): the rendering
 * stage of Sect. 3.1 (tile lists, then each tile's list drawn by the worker
 * that owns the tile's pixels, the image accumulated on the device), i.e. the
 * tiled splat, large-particle path, depth sort and finalisation of
 * spl_render, starting after the projection.  cam supplies width and height; prm supplies mode,
 * nu, tile, bin_rule, large_cut and normalise.  out: device image.  st may be
 * NULL (then the call does not synchronise at the end). */
spl_status spl_render_records(spl_ctx *ctx, int64_t n, const float *rec,
                              const float *rec2, const spl_camera *cam,
                              const spl_params *prm, float *out, spl_stats *st,
                              void *stream);

/* Full frame (Sect. 2.1: particles, camera and colour maps in, an RGB image
 * out; Sect. 3.1: rasterisation loops, then the tiled render): projection +
 * colour, tile binning, splat (small and large particle paths, or
 * depth-sorted compositing), finalisation.  p: device arrays the caller owns.
 * out: device image.  st may be NULL. */
spl_status spl_render(spl_ctx *ctx, const spl_particles *p, const spl_camera *cam,
                      const spl_params *prm, float *out, spl_stats *st, void *stream);

/* Resident data sets (Sect. 2.1: particle data are converted to the code's
 * internal format as they are read).  Copies src (host arrays when
 * src_on_device = 0, device arrays on the context's device when 1) into
 * device memory the data set owns, converting h, intensity, scalar and rgb to
 * store_dtype on the device: FP32 as is, BF16 rounded to nearest even, FP16
 * divided by a power of two per array (the one that puts the largest finite
 * magnitude in [2^10, 2^11)) and rounded to nearest even.  Positions,
 * species and absorption are copied as they are.  The data set lives on the
 * context's device until spl_dataset_free and may be used by every context
 * on that device (concurrent renders only read it).  Synchronises. */
spl_status spl_dataset_upload(spl_ctx *ctx, const spl_particles *src, int32_t src_on_device,
                              int32_t store_dtype, spl_dataset **out, void *stream);
void spl_dataset_free(spl_dataset *ds);
/* The resident arrays (device pointers, stored dtype and scales) for the
 * calls that take spl_particles.  The pointers stay valid until
 * spl_dataset_free. */
spl_status spl_dataset_particles(const spl_dataset *ds, spl_particles *out);
/* Device bytes the data set holds. */
int64_t spl_dataset_bytes(const spl_dataset *ds);

/* spl_render on a resident data set.  out_on_device = 1: out is a device
 * image; 0: out is host memory (height x width x 3 floats), filled from a
 * device image in the context workspace (Sect. 3.1: the image is copied back
 * to the host at the end), and the call synchronises. */
spl_status spl_render_dataset(spl_ctx *ctx, const spl_dataset *ds, const spl_camera *cam,
                              const spl_params *prm, float *out, int32_t out_on_device,
                              spl_stats *st, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the frame of
 * spl_render, with every workspace buffer taken from a fixed device array of
 * spl_noalloc_scratch_bytes() bytes (128 MiB) that the library holds on each
 * device until the process ends.  The call allocates nothing: no hipMalloc,
 * hipFree or allocating library routine; the context's own workspace is not
 * touched.  Inputs, output and stats as spl_render; stage timers are not
 * recorded.  Limits: a frame whose records, spans, tile lists and sort keys
 * do not fit returns SPL_ENOMEM with the sizes in spl_last_error.  Per
 * particle the frame needs 40 bytes (48 in sorted mode), checked before any
 * work is enqueued (at most about 3.3M and 2.8M particles); the lists, known
 * after the count, need 4 bytes per (particle, tile) entry (16 in sorted
 * mode, 8 in the deterministic additive order), so at 1.5 entries per
 * particle about 2.9M and 1.8M particles fit.
 * Every call on one device shares that device's array and finds the previous
 * call's contents there (the frame clears what must start at zero): calls
 * that overlap on one device, from any context, thread or stream, race and
 * must be serialised by the caller. */
spl_status spl_render_noalloc(spl_ctx *ctx, const spl_particles *p, const spl_camera *cam,
                              const spl_params *prm, float *out, spl_stats *st, void *stream);
int64_t spl_noalloc_scratch_bytes(void);

/* Many views of one resident particle set (the paper's scene-file frame
 * sequence, Sect. 2.1).  cams, prms, outs: host arrays of n_views entries
 * (outs[v] device images).  The projections, tile counts and scans of all
 * views are enqueued back to back before one host synchronisation reads all
 * list sizes; the splat of all views then runs as one persistent launch over
 * (view, tile-chunk) work items.  Views drawn in list order (SPL_SORTED, or
 * deterministic additive views) are rendered one after another as by
 * spl_render.  st: host array of n_views entries or NULL. */
spl_status spl_render_batch(spl_ctx *ctx, const spl_particles *p, int32_t n_views,
                            const spl_camera *cams, const spl_params *prms,
                            float *const *outs, spl_stats *st, void *stream);
/* spl_render_batch on a resident data set; outs[v] are device images when
 * out_on_device = 1, host memory when 0 (then the call synchronises). */
spl_status spl_render_batch_dataset(spl_ctx *ctx, const spl_dataset *ds, int32_t n_views,
                                    const spl_camera *cams, const spl_params *prms,
                                    float *const *outs, int32_t out_on_device, spl_stats *st,
                                    void *stream);

/* Out-of-core rendering (Sect. 3.1: data larger than the device memory are
 * copied in chunks into two device buffers, the next chunk copied while the
 * current one renders, and the image accumulates over the chunks before it
 * is copied back).  p: host arrays (attr_dtype any; memory from
 * spl_host_alloc lets the copies overlap the rendering, pageable memory
 * works without the overlap).  chunk: particles per chunk, >= 1; the two
 * buffers hold 2 x chunk particles.  The copies run on a second stream of
 * the context (default priority) ordered against `stream` by events.
 * Additive modes only: SPL_EUNSUPPORTED for SPL_SORTED (depth order spans
 * chunks).  The absorption = emission map and the normalisation apply once,
 * to the summed image.  out/out_on_device as spl_render_dataset; st sums the
 * particle and list counts over the chunks.  Synchronises. */
spl_status spl_render_stream(spl_ctx *ctx, const spl_particles *p, int64_t chunk,
                             const spl_camera *cam, const spl_params *prm, float *out,
                             int32_t out_on_device, spl_stats *st, void *stream);
/* Page-locked host memory for spl_render_stream's inputs. */
spl_status spl_host_alloc(size_t bytes, void **out);
void spl_host_free(void *p);

/* Tuning (Sect. 3.2.3: a script runs the code over candidate values of the
 * tile size and keeps the fastest).  Renders this view with tile sizes 16
 * and 32 and large-particle cuts 16, 32, 64, 128 px and none, timed on the
 * device, and caches the fastest choice for (n, width x height, mode, camera
 * pose): later frames of the same view with tile = 0 or large_cut = 0 take
 * it; other poses of the same size take the choice of the most recently
 * tuned pose.  tile and large_cut: host outputs.  Synchronises. */
spl_status spl_autotune(spl_ctx *ctx, const spl_particles *p, const spl_camera *cam,
                        const spl_params *prm, int32_t *tile, double *large_cut,
                        void *stream);

/* Stage timers.  When enabled, every frame records HIP events on its stream
 * around its stages; spl_get_timing returns, per stage, the summed device time
 * between the events and the summed algorithmic HBM bytes of the stage, over
 * all frames since the previous call, then resets.  Stages:
 *   0 projection + colour (or record spans), 1 tile counts, 2 scan,
 *   3 host gap + work-item build, 4 list scatter, 5 depth sort,
 *   6 image clear + large-particle splat, 7 tile splat / composite,
 *   8 finalise + FP64 reductions.
 * Algorithmic bytes count each array the stage must read or write once.
 * ms, bytes: host arrays of SPL_N_STAGES doubles.  Synchronises. */
#define SPL_N_STAGES 9
spl_status spl_set_timing(spl_ctx *ctx, int32_t enable);

/* Context options.
 *  SPL_OPT_TIMING       0/1: stage timers (same as spl_set_timing).
 *  SPL_OPT_GRAPHS       0/1: spl_render_batch records the launches after its
 *                       list-size synchronisation as a HIP graph and replays it.
 *  SPL_OPT_BATCH_BYTES  device bytes spl_render_batch may use for per-view
 *                       workspace; views beyond it go to later launches
 *                       (default 48 GiB).
 *  SPL_OPT_BATCH_PAIRS  tile-list entries one persistent splat launch of
 *                       spl_render_batch may hold (1 .. 2^32 - 2, the default);
 *                       views beyond it go to the next launch, which reuses
 *                       the list buffers.  A single view with more entries
 *                       is rendered alone. */
enum { SPL_OPT_TIMING = 0, SPL_OPT_GRAPHS = 1, SPL_OPT_BATCH_BYTES = 2, SPL_OPT_BATCH_PAIRS = 3 };
spl_status spl_set_option(spl_ctx *ctx, int32_t option, int64_t value);
spl_status spl_get_timing(spl_ctx *ctx, double *ms, double *bytes, int64_t *frames);

#ifdef __cplusplus
}
#endif
#endif
