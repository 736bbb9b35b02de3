/*
 * splref.c -- plain FP64 CPU oracle for the Splotch render pipeline.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product library.  Slow on
 * purpose: every loop is the definition written out, one particle and one
 * pixel at a time, in double precision.  No code is shared with the HIP path.
 *
 * Readings of the paper (Dykes et al., arXiv:1606.04427) used here; the paper
 * names these steps but prints no formula for them:
 *
 *  Camera (Sect. 2.1: particles are roto-translated and perspective-projected
 *  with respect to camera and look-at positions, then clipped).  Forward axis
 *  f = (lookat - eye)/|..|, right r = f x up/|..|, up' = r x f.  For
 *  v = p - eye: xv = v.r, yv = v.up', zv = v.f.  Focal length
 *  F = (H/2)/tan(fov_y/2).  X = W/2 + F xv/zv, Y = H/2 - F yv/zv (row 0 at the
 *  top).  Pixel (i, j) covers [i, i+1) x [j, j+1), centre (i+1/2, j+1/2).
 *
 *  Kernel (Sect. 2.1: the affected area follows the particle radius through a
 *  Gaussian kernel).  Projected radius rho = F h / zv; width
 *  sigma = sqrt((k_sigma rho)^2 + sigma_min^2); truncation radius
 *  R = nu sigma; column density tau = exp(-d^2/sigma^2) / (pi sigma^2) for
 *  d <= R (unit integral over the plane).
 *
 *  Clipping: a particle is active when its inputs are finite, h > 0, its
 *  species has a palette, zv > z_near, its centre and radius are within 2^22 px
 *  of the image and its pixel box meets the image.  In additive modes a
 *  particle with zero emission is dropped (it adds nothing); in sorted mode
 *  it stays if it absorbs.
 *
 *  Colour (Sect. 2.1: ranging, normalisation and an optional logarithm, then
 *  a colour map loaded at run time; Sect. 3.2.2: the colour stage walks an
 *  external look-up table).  g = log10(s) or s; t = clamp((g-lo)/(hi-lo), 0, 1)
 *  (t = 0 when hi = lo or when s <= 0 under the logarithm); linear
 *  interpolation between M evenly spaced entries; E = brightness * I * c.
 *  Sect. 2.1 also allows the colour to come directly from a vector field: a
 *  species with vector_colour takes c = the particle's own rgb vector (no
 *  ranging), and a particle whose vector has a non-finite component is
 *  inactive.
 *
 *  Radiative transfer (Sect. 2.1 refers to the transfer equation; Sect. 3.2.2
 *  describes additive drawing).  Per particle slab with optical depth
 *  x = a tau: I_out = I_in exp(-x) + E tau phi(x), phi(x) = (1-exp(-x))/x.
 *   - ADD_RAW:  J = sum_p E_p tau_p (the additive drawing rule).
 *   - ADD_AEQE: absorption equal to emission, I = 1 - exp(-J), exact solution
 *     of dI/ds = E rho (1 - I), independent of order.
 *   - SORTED:   separate absorption; particles composited in ascending view
 *     depth, front to back: C += T E tau phi(x), T *= exp(-x).  The depth used
 *     for ordering is rounded to single precision and ties go by particle
 *     index (the paper fixes no order for particles at equal depth).
 *
 *  Tiles (Sect. 3.1; tile-list pseudocode figure): the image is cut in square
 *  tiles of T px; a particle is listed in every tile its pixel box touches.
 *  The paper's own rule keeps a tile only if the distance from the particle
 *  to the tile centre is below 0.75 radius + sqrt(2) T/2 (Fig. "tilesdiagram"
 *  drops a corner overlap as negligible); it is available as bin_rule 1.
 */
#include "splref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define SR_PI 3.14159265358979323846
#define SR_RANGE_LIMIT 4194304.0 /* 2^22 px */

static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

static int finite3(const double *v) {
  return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

int sr_frame(const sr_camera *cam, double out[13]) {
  double f[3], r[3], u[3], n;
  int k;
  if (!cam) return SR_EINVAL;
  if (cam->width < 1 || cam->height < 1 || cam->width > 32768 ||
      cam->height > 32768)
    return SR_EINVAL;
  if (!(cam->fov_y_deg > 0.0 && cam->fov_y_deg < 180.0)) return SR_EINVAL;
  if (!(cam->z_near >= 0.0) || !isfinite(cam->z_near)) return SR_EINVAL;
  if (!finite3(cam->eye) || !finite3(cam->lookat) || !finite3(cam->up))
    return SR_EINVAL;
  for (k = 0; k < 3; ++k) f[k] = cam->lookat[k] - cam->eye[k];
  n = sqrt(dot3(f, f));
  if (!(n > 0.0)) return SR_EINVAL;
  for (k = 0; k < 3; ++k) f[k] /= n;
  cross3(f, cam->up, r);
  n = sqrt(dot3(r, r));
  if (!(n > 1e-12)) return SR_EINVAL; /* up parallel to the view direction */
  for (k = 0; k < 3; ++k) r[k] /= n;
  cross3(r, f, u);
  for (k = 0; k < 3; ++k) {
    out[k] = cam->eye[k];
    out[3 + k] = r[k];
    out[6 + k] = u[k];
    out[9 + k] = f[k];
  }
  out[12] = 0.5 * (double)cam->height / tan(0.5 * cam->fov_y_deg * SR_PI / 180.0);
  return SR_OK;
}

int sr_validate(const sr_camera *cam, const sr_params *prm) {
  double fr[13];
  int k;
  if (sr_frame(cam, fr) != SR_OK) return SR_EINVAL;
  if (!prm) return SR_EINVAL;
  if (prm->mode < SR_ADD_RAW || prm->mode > SR_SORTED) return SR_EINVAL;
  if (prm->n_species < 1 || prm->n_species > 256 || !prm->looks) return SR_EINVAL;
  if (!(prm->k_sigma >= 0.0) || !isfinite(prm->k_sigma)) return SR_EINVAL;
  if (!(prm->sigma_min > 0.0) || !isfinite(prm->sigma_min)) return SR_EINVAL;
  if (!(prm->nu > 0.0) || !isfinite(prm->nu)) return SR_EINVAL;
  for (k = 0; k < prm->n_species; ++k) {
    const sr_look *l = &prm->looks[k];
    if (l->vector_colour) continue; /* no palette is read */
    if (!l->rgb || l->n_entries < 1) return SR_EINVAL;
    if (!isfinite(l->lo) || !isfinite(l->hi) || !(l->hi >= l->lo)) return SR_EINVAL;
    if (!isfinite(l->brightness)) return SR_EINVAL;
  }
  return SR_OK;
}

/* Normalised scalar t in [0, 1] (ranging + normalisation + optional log). */
static double normalise_scalar(double s, const sr_look *l) {
  double g, t;
  if (l->log10_scalar) {
    if (!(s > 0.0)) return 0.0;
    g = log10(s);
  } else {
    g = s;
  }
  if (l->hi == l->lo) return 0.0;
  t = (g - l->lo) / (l->hi - l->lo);
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  return t;
}

/* Colour map: linear interpolation between evenly spaced entries. */
static void palette_lookup(const sr_look *l, double t, double c[3]) {
  int M = l->n_entries, j, k;
  double u, f;
  if (M == 1) {
    for (k = 0; k < 3; ++k) c[k] = (double)l->rgb[k];
    return;
  }
  u = t * (double)(M - 1);
  j = (int)floor(u);
  if (j > M - 2) j = M - 2;
  if (j < 0) j = 0;
  f = u - (double)j;
  for (k = 0; k < 3; ++k)
    c[k] = (1.0 - f) * (double)l->rgb[3 * j + k] + f * (double)l->rgb[3 * (j + 1) + k];
}

/* Projects particle k.  *valid = passes every test except the image overlap
 * (used by the brute-force renderer, which has no pixel box). */
static void project_one(const double fr[13], const sr_camera *cam,
                        const sr_params *prm, const sr_particles *p, int64_t k,
                        sr_proj *o, int *valid) {
  double v[3], c[3], xv, yv, zv, F = fr[12], ks;
  double x = p->x[k], y = p->y[k], z = p->z[k], h = p->h[k];
  double I = p->intensity[k], s = p->scalar[k];
  double a = (prm->mode == SR_SORTED && p->absorption) ? p->absorption[k] : 0.0;
  int sp = p->species ? (int)p->species[k] : 0;
  const sr_look *l;
  int q;
  memset(o, 0, sizeof(*o));
  *valid = 0;
  if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(h) &&
        isfinite(I) && isfinite(s) && isfinite(a)))
    return;
  if (!(h > 0.0) || sp >= prm->n_species || a < 0.0) return;
  v[0] = x - fr[0];
  v[1] = y - fr[1];
  v[2] = z - fr[2];
  xv = dot3(v, fr + 3);
  yv = dot3(v, fr + 6);
  zv = dot3(v, fr + 9);
  if (!(zv > cam->z_near)) return;
  o->zv = zv;
  o->X = 0.5 * cam->width + F * xv / zv;
  o->Y = 0.5 * cam->height - F * yv / zv;
  o->rho = F * h / zv;
  ks = prm->k_sigma * o->rho;
  o->sigma = sqrt(ks * ks + prm->sigma_min * prm->sigma_min);
  o->R = prm->nu * o->sigma;
  if (!(fabs(o->X - 0.5 * cam->width) <= SR_RANGE_LIMIT &&
        fabs(o->Y - 0.5 * cam->height) <= SR_RANGE_LIMIT &&
        o->R <= SR_RANGE_LIMIT))
    return;
  l = &prm->looks[sp];
  if (l->vector_colour) {
    for (q = 0; q < 3; ++q) c[q] = p->rgb[3 * k + q];
    if (!(isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]))) return;
  } else {
    palette_lookup(l, normalise_scalar(s, l), c);
  }
  for (q = 0; q < 3; ++q) o->E[q] = l->brightness * I * c[q];
  o->a = a;
  if (prm->mode != SR_SORTED) {
    if (o->E[0] == 0.0 && o->E[1] == 0.0 && o->E[2] == 0.0) return;
  } else {
    if (o->E[0] == 0.0 && o->E[1] == 0.0 && o->E[2] == 0.0 && a == 0.0) return;
  }
  *valid = 1;
  /* pixel box: centres i + 1/2 within [X - R, X + R] */
  {
    double i0 = ceil(o->X - o->R - 0.5), i1 = floor(o->X + o->R - 0.5);
    double j0 = ceil(o->Y - o->R - 0.5), j1 = floor(o->Y + o->R - 0.5);
    if (i0 < 0.0) i0 = 0.0;
    if (j0 < 0.0) j0 = 0.0;
    if (i1 > cam->width - 1) i1 = cam->width - 1;
    if (j1 > cam->height - 1) j1 = cam->height - 1;
    if (i0 > i1 || j0 > j1) return;
    o->i0 = (int32_t)i0;
    o->i1 = (int32_t)i1;
    o->j0 = (int32_t)j0;
    o->j1 = (int32_t)j1;
    o->active = 1;
  }
}

int sr_project(const sr_particles *p, const sr_camera *cam,
               const sr_params *prm, sr_proj *out) {
  double fr[13];
  int64_t k;
  int valid;
  if (sr_validate(cam, prm) != SR_OK || !p || p->n < 0 || !out) return SR_EINVAL;
  if (p->n > 0 && (!p->x || !p->y || !p->z || !p->h || !p->intensity || !p->scalar))
    return SR_EINVAL;
  if (prm->mode == SR_SORTED && p->n > 0 && !p->absorption) return SR_EINVAL;
  for (k = 0; k < prm->n_species; ++k)
    if (prm->looks[k].vector_colour && p->n > 0 && !p->rgb) return SR_EINVAL;
  sr_frame(cam, fr);
  for (k = 0; k < p->n; ++k) project_one(fr, cam, prm, p, k, &out[k], &valid);
  return SR_OK;
}

int sr_expected_flux(const sr_particles *p, const sr_camera *cam,
                     const sr_params *prm, double expected[3]) {
  sr_proj *pr;
  int64_t k;
  int rc, q;
  if (!p || p->n < 0 || !expected) return SR_EINVAL;
  if (sr_validate(cam, prm) != SR_OK || prm->mode == SR_SORTED) return SR_EINVAL;
  pr = (sr_proj *)malloc(sizeof(sr_proj) * (p->n > 0 ? p->n : 1));
  if (!pr) return SR_ENOMEM;
  rc = sr_project(p, cam, prm, pr);
  if (rc != SR_OK) {
    free(pr);
    return rc;
  }
  for (q = 0; q < 3; ++q) expected[q] = 0.0;
  for (k = 0; k < p->n; ++k) {
    const sr_proj *o = &pr[k];
    double kappa = 0.0, R2 = o->R * o->R, amp;
    int i, j;
    if (!o->active) continue;
    amp = 1.0 / (SR_PI * o->sigma * o->sigma);
    for (j = o->j0; j <= o->j1; ++j)
      for (i = o->i0; i <= o->i1; ++i) {
        double dx = i + 0.5 - o->X, dy = j + 0.5 - o->Y, d2 = dx * dx + dy * dy;
        if (d2 <= R2) kappa += amp * exp(-d2 / (o->sigma * o->sigma));
      }
    for (q = 0; q < 3; ++q) expected[q] += o->E[q] * kappa;
  }
  free(pr);
  return SR_OK;
}

int sr_scalar_range(const sr_particles *p, int32_t n_species,
                    int32_t log10_scalar, double *lo, double *hi) {
  int64_t k;
  int sp;
  if (!p || p->n < 0 || n_species < 1 || !lo || !hi) return SR_EINVAL;
  if (p->n > 0 && !p->scalar) return SR_EINVAL;
  for (sp = 0; sp < n_species; ++sp) {
    lo[sp] = INFINITY;
    hi[sp] = -INFINITY;
  }
  for (k = 0; k < p->n; ++k) {
    double s = p->scalar[k], g;
    sp = p->species ? (int)p->species[k] : 0;
    if (sp >= n_species || !isfinite(s)) continue;
    if (log10_scalar) {
      if (!(s > 0.0)) continue;
      g = log10(s);
    } else {
      g = s;
    }
    if (g < lo[sp]) lo[sp] = g;
    if (g > hi[sp]) hi[sp] = g;
  }
  return SR_OK;
}

static double phi_slab(double x) {
  /* (1 - exp(-x)) / x, with its series below 1e-8 */
  if (x < 1e-8) return 1.0 - 0.5 * x;
  return -expm1(-x) / x;
}

typedef struct {
  double key;
  int64_t idx;
} depth_item;

static int cmp_depth(const void *a, const void *b) {
  const depth_item *x = (const depth_item *)a, *y = (const depth_item *)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->idx > y->idx) - (x->idx < y->idx);
}

static void normalise_by_max(double *out, int64_t n) {
  double m = 0.0;
  int64_t k;
  for (k = 0; k < n; ++k)
    if (out[k] > m) m = out[k];
  if (m > 0.0)
    for (k = 0; k < n; ++k) out[k] /= m;
}

static int render_impl(const sr_particles *p, const sr_camera *cam,
                       const sr_params *prm, double *out, int back_to_front) {
  int64_t npx, k;
  sr_proj *pr;
  int rc;
  if (!out) return SR_EINVAL;
  if (sr_validate(cam, prm) != SR_OK) return SR_EINVAL;
  npx = (int64_t)cam->width * cam->height;
  memset(out, 0, sizeof(double) * 3 * npx);
  pr = (sr_proj *)malloc(sizeof(sr_proj) * (p->n > 0 ? p->n : 1));
  if (!pr) return SR_ENOMEM;
  rc = sr_project(p, cam, prm, pr);
  if (rc != SR_OK) {
    free(pr);
    return rc;
  }
  if (prm->mode != SR_SORTED) {
    for (k = 0; k < p->n; ++k) {
      const sr_proj *o = &pr[k];
      int i, j, q;
      double amp, R2;
      if (!o->active) continue;
      amp = 1.0 / (SR_PI * o->sigma * o->sigma);
      R2 = o->R * o->R;
      for (j = o->j0; j <= o->j1; ++j)
        for (i = o->i0; i <= o->i1; ++i) {
          double dx = i + 0.5 - o->X, dy = j + 0.5 - o->Y;
          double d2 = dx * dx + dy * dy, tau;
          if (d2 > R2) continue;
          tau = amp * exp(-d2 / (o->sigma * o->sigma));
          for (q = 0; q < 3; ++q) out[3 * ((int64_t)j * cam->width + i) + q] += o->E[q] * tau;
        }
    }
    if (prm->mode == SR_ADD_AEQE)
      for (k = 0; k < 3 * npx; ++k) out[k] = -expm1(-out[k]);
  } else {
    depth_item *ord;
    double *T = NULL;
    int64_t na = 0, m;
    ord = (depth_item *)malloc(sizeof(depth_item) * (p->n > 0 ? p->n : 1));
    if (!back_to_front) T = (double *)malloc(sizeof(double) * (npx > 0 ? npx : 1));
    if (!ord || (!back_to_front && !T)) {
      free(ord);
      free(T);
      free(pr);
      return SR_ENOMEM;
    }
    /* Depth order: view depth rounded to single precision, ties by index.
     * Two depths within one single-precision step (~1e-7 relative) have no
     * physically meaningful order; this fixes one. */
    for (k = 0; k < p->n; ++k)
      if (pr[k].active) {
        ord[na].key = (double)(float)pr[k].zv;
        ord[na].idx = k;
        ++na;
      }
    qsort(ord, (size_t)na, sizeof(depth_item), cmp_depth);
    if (!back_to_front)
      for (k = 0; k < npx; ++k) T[k] = 1.0;
    for (m = 0; m < na; ++m) {
      const sr_proj *o = &pr[back_to_front ? ord[na - 1 - m].idx : ord[m].idx];
      double amp = 1.0 / (SR_PI * o->sigma * o->sigma), R2 = o->R * o->R;
      int i, j, q;
      for (j = o->j0; j <= o->j1; ++j)
        for (i = o->i0; i <= o->i1; ++i) {
          double dx = i + 0.5 - o->X, dy = j + 0.5 - o->Y;
          double d2 = dx * dx + dy * dy, tau, x, ph;
          int64_t pix = (int64_t)j * cam->width + i;
          if (d2 > R2) continue;
          tau = amp * exp(-d2 / (o->sigma * o->sigma));
          x = o->a * tau;
          ph = phi_slab(x);
          if (!back_to_front) {
            for (q = 0; q < 3; ++q) out[3 * pix + q] += T[pix] * o->E[q] * tau * ph;
            T[pix] *= exp(-x);
          } else {
            for (q = 0; q < 3; ++q)
              out[3 * pix + q] = out[3 * pix + q] * exp(-x) + o->E[q] * tau * ph;
          }
        }
    }
    free(ord);
    free(T);
  }
  if (prm->normalise) normalise_by_max(out, 3 * npx);
  free(pr);
  return SR_OK;
}

int sr_render(const sr_particles *p, const sr_camera *cam,
              const sr_params *prm, double *out) {
  if (!p || p->n < 0) return SR_EINVAL;
  return render_impl(p, cam, prm, out, 0);
}

int sr_render_sorted_back_to_front(const sr_particles *p, const sr_camera *cam,
                                   const sr_params *prm, double *out) {
  if (!p || p->n < 0 || !prm || prm->mode != SR_SORTED) return SR_EINVAL;
  return render_impl(p, cam, prm, out, 1);
}

int sr_render_brute(const sr_particles *p, const sr_camera *cam,
                    const sr_params *prm, int32_t truncate, double *out) {
  double fr[13];
  int64_t npx, k;
  int i, j, q, valid;
  sr_proj o;
  if (!p || p->n < 0 || !out) return SR_EINVAL;
  if (sr_validate(cam, prm) != SR_OK || prm->mode == SR_SORTED) return SR_EINVAL;
  if (p->n > 0 && (!p->x || !p->y || !p->z || !p->h || !p->intensity || !p->scalar))
    return SR_EINVAL;
  for (k = 0; k < prm->n_species; ++k)
    if (prm->looks[k].vector_colour && p->n > 0 && !p->rgb) return SR_EINVAL;
  sr_frame(cam, fr);
  npx = (int64_t)cam->width * cam->height;
  memset(out, 0, sizeof(double) * 3 * npx);
  for (k = 0; k < p->n; ++k) {
    double amp, R2;
    project_one(fr, cam, prm, p, k, &o, &valid);
    if (!valid) continue;
    amp = 1.0 / (SR_PI * o.sigma * o.sigma);
    R2 = o.R * o.R;
    for (j = 0; j < cam->height; ++j)
      for (i = 0; i < cam->width; ++i) {
        double dx = i + 0.5 - o.X, dy = j + 0.5 - o.Y, d2 = dx * dx + dy * dy, tau;
        if (truncate && d2 > R2) continue;
        tau = amp * exp(-d2 / (o.sigma * o.sigma));
        for (q = 0; q < 3; ++q) out[3 * ((int64_t)j * cam->width + i) + q] += o.E[q] * tau;
      }
  }
  if (prm->mode == SR_ADD_AEQE)
    for (k = 0; k < 3 * npx; ++k) out[k] = -expm1(-out[k]);
  if (prm->normalise) normalise_by_max(out, 3 * npx);
  return SR_OK;
}

/* ---------------- single-precision records ------------------------------ */

int sr_record_box(const float *rec, float nu, int32_t width, int32_t height,
                  int32_t *i0, int32_t *i1, int32_t *j0, int32_t *j1) {
  /* Every operation below is one IEEE single-precision operation in the
   * order written; the file is compiled without contraction. */
  float Xi = rec[0], Xf = rec[1], Yi = rec[2], Yf = rec[3], s = rec[4];
  float R, fx, fy, lx, hx, ly, hy;
  double a0, a1, b0, b1;
  if (!(s > 0.0f)) return 0;
  if (!(isfinite(Xi) && isfinite(Xf) && isfinite(Yi) && isfinite(Yf) && isfinite(s)))
    return 0;
  R = nu * s;
  fx = Xf - 0.5f;
  fy = Yf - 0.5f;
  lx = fx - R;
  hx = fx + R;
  ly = fy - R;
  hy = fy + R;
  a0 = (double)Xi + (double)ceilf(lx);
  a1 = (double)Xi + (double)floorf(hx);
  b0 = (double)Yi + (double)ceilf(ly);
  b1 = (double)Yi + (double)floorf(hy);
  if (a0 < 0.0) a0 = 0.0;
  if (b0 < 0.0) b0 = 0.0;
  if (a1 > width - 1) a1 = width - 1;
  if (b1 > height - 1) b1 = height - 1;
  if (a0 > a1 || b0 > b1) return 0;
  *i0 = (int32_t)a0;
  *i1 = (int32_t)a1;
  *j0 = (int32_t)b0;
  *j1 = (int32_t)b1;
  return 1;
}

/* The paper's tile-inclusion threshold, in single precision. */
static int paper_rule_keeps(const float *rec, float nu, int32_t tile, int32_t tx,
                            int32_t ty) {
  float R = nu * rec[4];
  float cx = (float)(tx * tile) + 0.5f * (float)tile;
  float cy = (float)(ty * tile) + 0.5f * (float)tile;
  float dx = (rec[0] - cx) + rec[1];
  float dy = (rec[2] - cy) + rec[3];
  float t1 = dx * dx, t2 = dy * dy, d2 = t1 + t2;
  float a1 = 0.75f * R, a2 = (float)tile * 0.70710678f, thr = a1 + a2;
  float thr2 = thr * thr;
  return d2 < thr2;
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

int sr_bin_records(int64_t n, const float *rec, const float *rec2,
                   int32_t width, int32_t height, int32_t tile, float nu,
                   int32_t bin_rule, int32_t by_depth, uint32_t *counts,
                   uint32_t *offsets, uint32_t *pairs, int64_t pairs_cap,
                   int64_t *n_pairs) {
  int32_t ntx, nty, i0, i1, j0, j1, tx, ty;
  int64_t nt, k, total = 0, t;
  uint32_t *cursor;
  if (n < 0 || (n > 0 && !rec) || width < 1 || height < 1 || tile < 1 || !counts ||
      !offsets || !n_pairs || (by_depth && n > 0 && !rec2))
    return SR_EINVAL;
  ntx = (width + tile - 1) / tile;
  nty = (height + tile - 1) / tile;
  nt = (int64_t)ntx * nty;
  memset(counts, 0, sizeof(uint32_t) * nt);
  for (k = 0; k < n; ++k) {
    const float *r = rec + 8 * k;
    if (!sr_record_box(r, nu, width, height, &i0, &i1, &j0, &j1)) continue;
    for (ty = j0 / tile; ty <= j1 / tile; ++ty)
      for (tx = i0 / tile; tx <= i1 / tile; ++tx)
        if (bin_rule == 0 || paper_rule_keeps(r, nu, tile, tx, ty))
          counts[(int64_t)ty * ntx + tx] += 1;
  }
  for (t = 0; t < nt; ++t) {
    offsets[t] = (uint32_t)total;
    total += counts[t];
  }
  offsets[nt] = (uint32_t)total;
  *n_pairs = total;
  if (!pairs) return SR_OK;
  if (total > pairs_cap) return SR_ENOMEM;
  cursor = (uint32_t *)malloc(sizeof(uint32_t) * (nt > 0 ? nt : 1));
  if (!cursor) return SR_ENOMEM;
  memcpy(cursor, offsets, sizeof(uint32_t) * nt);
  for (k = 0; k < n; ++k) {
    const float *r = rec + 8 * k;
    if (!sr_record_box(r, nu, width, height, &i0, &i1, &j0, &j1)) continue;
    for (ty = j0 / tile; ty <= j1 / tile; ++ty)
      for (tx = i0 / tile; tx <= i1 / tile; ++tx)
        if (bin_rule == 0 || paper_rule_keeps(r, nu, tile, tx, ty))
          pairs[cursor[(int64_t)ty * ntx + tx]++] = (uint32_t)k;
  }
  free(cursor);
  if (by_depth) {
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (total > 0 ? total : 1));
    if (!keys) return SR_ENOMEM;
    for (t = 0; t < nt; ++t) {
      int64_t b = offsets[t], e = offsets[t + 1], m;
      for (m = b; m < e; ++m) {
        uint32_t bits;
        memcpy(&bits, &rec2[2 * (int64_t)pairs[m] + 1], 4);
        keys[m - b] = ((uint64_t)bits << 32) | pairs[m];
      }
      qsort(keys, (size_t)(e - b), sizeof(uint64_t), cmp_u64);
      for (m = b; m < e; ++m) pairs[m] = (uint32_t)(keys[m - b] & 0xffffffffu);
    }
    free(keys);
  }
  return SR_OK;
}

int sr_render_records(int64_t n, const float *rec, const float *rec2,
                      int32_t width, int32_t height, int32_t mode, double nu,
                      double *out) {
  int64_t npx = (int64_t)width * height, k;
  int32_t i0, i1, j0, j1, i, j, q;
  if (n < 0 || (n > 0 && !rec) || width < 1 || height < 1 || !out) return SR_EINVAL;
  if (mode < SR_ADD_RAW || mode > SR_SORTED || !(nu > 0.0)) return SR_EINVAL;
  if (mode == SR_SORTED && n > 0 && !rec2) return SR_EINVAL;
  memset(out, 0, sizeof(double) * 3 * npx);
  if (mode != SR_SORTED) {
    for (k = 0; k < n; ++k) {
      const float *r = rec + 8 * k;
      double X, Y, s, R2;
      if (!sr_record_box(r, (float)nu, width, height, &i0, &i1, &j0, &j1)) continue;
      X = (double)r[0] + (double)r[1];
      Y = (double)r[2] + (double)r[3];
      s = (double)r[4];
      R2 = (nu * s) * (nu * s);
      for (j = j0; j <= j1; ++j)
        for (i = i0; i <= i1; ++i) {
          double dx = i + 0.5 - X, dy = j + 0.5 - Y, d2 = dx * dx + dy * dy, g;
          if (d2 > R2) continue;
          g = exp(-d2 / (s * s));
          for (q = 0; q < 3; ++q) out[3 * ((int64_t)j * width + i) + q] += (double)r[5 + q] * g;
        }
    }
    if (mode == SR_ADD_AEQE)
      for (k = 0; k < 3 * npx; ++k) out[k] = -expm1(-out[k]);
  } else {
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
    double *T = (double *)malloc(sizeof(double) * (npx > 0 ? npx : 1));
    int64_t na = 0, m;
    if (!keys || !T) {
      free(keys);
      free(T);
      return SR_ENOMEM;
    }
    for (k = 0; k < n; ++k) {
      uint32_t bits;
      if (!sr_record_box(rec + 8 * k, (float)nu, width, height, &i0, &i1, &j0, &j1))
        continue;
      memcpy(&bits, &rec2[2 * k + 1], 4);
      keys[na++] = ((uint64_t)bits << 32) | (uint64_t)k;
    }
    qsort(keys, (size_t)na, sizeof(uint64_t), cmp_u64);
    for (k = 0; k < npx; ++k) T[k] = 1.0;
    for (m = 0; m < na; ++m) {
      int64_t p = (int64_t)(keys[m] & 0xffffffffu);
      const float *r = rec + 8 * p;
      double X = (double)r[0] + (double)r[1], Y = (double)r[2] + (double)r[3];
      double s = (double)r[4], R2 = (nu * s) * (nu * s), ap = (double)rec2[2 * p];
      sr_record_box(r, (float)nu, width, height, &i0, &i1, &j0, &j1);
      for (j = j0; j <= j1; ++j)
        for (i = i0; i <= i1; ++i) {
          double dx = i + 0.5 - X, dy = j + 0.5 - Y, d2 = dx * dx + dy * dy, g, x, ph;
          int64_t pix = (int64_t)j * width + i;
          if (d2 > R2) continue;
          g = exp(-d2 / (s * s));
          x = ap * g;
          ph = phi_slab(x);
          for (q = 0; q < 3; ++q) out[3 * pix + q] += T[pix] * (double)r[5 + q] * g * ph;
          T[pix] *= exp(-x);
        }
    }
    free(keys);
    free(T);
  }
  return SR_OK;
}

void sr_image_stats(const double *img, int32_t width, int32_t height,
                    double flux[3], double maxv[3]) {
  int64_t npx = (int64_t)width * height, k;
  int q;
  for (q = 0; q < 3; ++q) {
    flux[q] = 0.0;
    maxv[q] = -INFINITY;
  }
  for (k = 0; k < npx; ++k)
    for (q = 0; q < 3; ++q) {
      double v = img[3 * k + q];
      flux[q] += v;
      if (v > maxv[q]) maxv[q] = v;
    }
}
