/*
 * splref.h -- plain FP64 CPU oracle for the Splotch render pipeline.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no source, header or helper with the
 * HIP path.
 *
 * Paper: Dykes, Gheller, Rivi, Krokos, "Splotch: porting and optimizing for the
 * Xeon Phi" (arXiv:1606.04427).  The paper names the stages of the method
 * (Sect. 2.1 "The Splotch Code"; Sect. 3.1 "Implementation") but prints no
 * equation; every formula below is a stated reading of those passages:
 *
 *  - preprocessing: ranging, normalisation, optional logarithm (Sect. 2.1)
 *  - rasterisation: roto-translation, perspective projection with respect to
 *    camera and look-at positions, clipping (Sect. 2.1, Sect. 3.1)
 *  - colour from a scalar field through a colour map loaded at run time, RGB
 *    as single-precision triplets (Sect. 2.1)
 *  - render: Gaussian kernel whose extent follows the particle radius
 *    (Sect. 2.1), contributions combined by the radiative-transfer equation;
 *    additive drawing = pixel + colour x scalar contribution (Sect. 3.2.2)
 *  - image split in square tiles with a particle list per tile (Sect. 3.1,
 *    Fig. "tilesdiagram" and the tile-list pseudocode figure).
 */
#ifndef SPLREF_H
#define SPLREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SR_ADD_RAW = 0, SR_ADD_AEQE = 1, SR_SORTED = 2 };
enum { SR_OK = 0, SR_EINVAL = -1, SR_ENOMEM = -2 };

typedef struct {
  double eye[3], lookat[3], up[3];
  double fov_y_deg; /* vertical field of view, degrees, in (0, 180) */
  double z_near;    /* particles with view depth <= z_near are clipped */
  int32_t width, height;
} sr_camera;

typedef struct {
  const float *rgb;     /* n_entries x 3, row-major, host memory */
  int32_t n_entries;    /* >= 1 */
  int32_t log10_scalar; /* 1: normalise log10(scalar) instead of scalar */
  double brightness;    /* multiplies every emission of the species */
  double lo, hi;        /* normalisation range of the (log) scalar, hi >= lo */
  int32_t vector_colour; /* 1: colour = the particle's rgb vector, no palette */
} sr_look;

typedef struct {
  int32_t mode;      /* SR_ADD_RAW, SR_ADD_AEQE or SR_SORTED */
  int32_t n_species; /* number of entries in looks, >= 1 */
  const sr_look *looks;
  double k_sigma;    /* sigma = sqrt((k_sigma * rho)^2 + sigma_min^2) */
  double sigma_min;  /* px */
  double nu;         /* truncation radius R = nu * sigma */
  int32_t normalise; /* 1: divide the output by its maximum value */
} sr_params;

typedef struct {
  int64_t n;
  const double *x, *y, *z;   /* world positions */
  const double *h;           /* smoothing length (world units) */
  const double *intensity;   /* scalar multiplying the colour */
  const double *scalar;      /* scalar field mapped through the palette */
  const double *absorption;  /* per-particle absorption; SR_SORTED only */
  const uint8_t *species;    /* may be NULL: every particle is species 0 */
  const double *rgb;         /* n x 3 colour vectors; needed by vector_colour */
} sr_particles;

/* Per-particle result of transform, projection, clipping and colour. */
typedef struct {
  double X, Y;     /* screen position, px; pixel (i, j) covers [i,i+1)x[j,j+1) */
  double zv;       /* view-space depth */
  double rho;      /* projected smoothing length, px */
  double sigma, R; /* kernel width and truncation radius, px */
  double E[3];     /* emission colour */
  double a;        /* absorption (0 in additive modes) */
  int32_t active;
  int32_t i0, i1, j0, j1; /* pixel bounding box of the disc, clipped */
} sr_proj;

/* Camera frame: out[0..2] eye, [3..5] right, [6..8] up, [9..11] forward,
 * [12] focal length in px.  Returns SR_EINVAL for a degenerate camera. */
int sr_frame(const sr_camera *cam, double out[13]);

/* Validates camera and parameters (same rules as the render calls). */
int sr_validate(const sr_camera *cam, const sr_params *prm);

/* Transform + project + clip + colour, one sr_proj per particle. */
int sr_project(const sr_particles *p, const sr_camera *cam,
               const sr_params *prm, sr_proj *out);

/* Ranging: per-species min and max of the (log10) scalar over finite values
 * (values <= 0 are skipped under log10).  lo/hi get +inf/-inf for a species
 * with no usable value. */
int sr_scalar_range(const sr_particles *p, int32_t n_species,
                    int32_t log10_scalar, double *lo, double *hi);

/* Full render in FP64: out is height x width x 3, row 0 = top. */
int sr_render(const sr_particles *p, const sr_camera *cam,
              const sr_params *prm, double *out);

/* Same image computed by visiting every pixel for every particle, without
 * bounding boxes.  truncate = 0 drops the R cut-off (untruncated Gaussian).
 * Additive modes only. */
int sr_render_brute(const sr_particles *p, const sr_camera *cam,
                    const sr_params *prm, int32_t truncate, double *out);

/* SR_SORTED only: composite from back to front instead of front to back. */
int sr_render_sorted_back_to_front(const sr_particles *p, const sr_camera *cam,
                                   const sr_params *prm, double *out);

/* ---- checks on single-precision projected records ----------------------
 * A record holds 8 floats {Xi, Xf, Yi, Yf, sigma, Ar, Ag, Ab}: the screen
 * position split into an integer part and a fraction (X = Xi + Xf), the
 * kernel width, and the colour premultiplied by the kernel amplitude
 * 1/(pi sigma^2).  sigma <= 0 marks an inactive particle.  rec2 (optional,
 * sorted mode) holds 2 floats {a * amplitude, zv} per particle. */

/* Pixel box of a record in single precision, clipped to the image.
 * Returns 1 if the clipped box is non-empty. */
int sr_record_box(const float *rec, float nu, int32_t width, int32_t height,
                  int32_t *i0, int32_t *i1, int32_t *j0, int32_t *j1);

/* Tile lists from records (single-precision rule).  tile = tile edge in px;
 * bin_rule 0 = every tile the pixel box touches, 1 = the paper's distance
 * threshold (0.75 * radius + sqrt(2) * tile / 2 from the tile centre, the
 * radius being the truncation radius R) applied inside that tile range.
 * counts: n_tiles; offsets: n_tiles + 1; pairs: particle indices, ascending
 * within each tile, or ascending (zv bits, index) when by_depth = 1 (needs
 * rec2).  pairs may be NULL to count only.  Returns SR_ENOMEM if pairs_cap is
 * too small (n_pairs is still set). */
int sr_bin_records(int64_t n, const float *rec, const float *rec2,
                   int32_t width, int32_t height, int32_t tile, float nu,
                   int32_t bin_rule, int32_t by_depth, uint32_t *counts,
                   uint32_t *offsets, uint32_t *pairs, int64_t pairs_cap,
                   int64_t *n_pairs);

/* Render from records in FP64 (inputs widened exactly).  mode as above;
 * sorted mode visits particles in ascending (zv bits, index) order. */
int sr_render_records(int64_t n, const float *rec, const float *rec2,
                      int32_t width, int32_t height, int32_t mode, double nu,
                      double *out);

/* Expected flux of the additive transfer sum: sum over active particles of
 * E_p kappa_p, kappa_p = sum over the pixels of the particle's clipped box
 * whose centres lie within R of tau_p (the sampled, truncated, clipped
 * kernel).  expected[3] per channel. */
int sr_expected_flux(const sr_particles *p, const sr_camera *cam,
                     const sr_params *prm, double expected[3]);

/* Image statistics: per-channel sum and maximum. */
void sr_image_stats(const double *img, int32_t width, int32_t height,
                    double flux[3], double maxv[3]);

#ifdef __cplusplus
}
#endif
#endif
