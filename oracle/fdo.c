/*
 * fdo.c -- CPU oracle for fusion-patch multi-view direction optimisation.
 *
 * TEST INFRASTRUCTURE ONLY (see fdo.h).  Plain loops in binary64, one point
 * at a time, no tiling, no reformulation of the paper's expressions.
 *
 * Build: gcc -O2 -std=c99 -fopenmp -ffp-contract=off -fPIC -shared.
 * Floating-point contraction stays off, so every expression below is
 * evaluated exactly as written (one rounding per operation).
 */
#define _POSIX_C_SOURCE 200809L
#include "fdo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define FDO_MAX_K 16
#define FDO_MAX_P 7
#define FDO_MAX_S 16
#define FDO_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* map access                                                                */

float fdo_half_to_float(uint16_t h) {
  uint32_t s = (h >> 15) & 1u, e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
  float v;
  if (e == 0)
    v = ldexpf((float)m, -24);
  else if (e == 31)
    v = m ? NAN : INFINITY;
  else
    v = ldexpf((float)(m | 0x400u), (int)e - 25);
  return s ? -v : v;
}

/* Texel (x, y) of one H x W map; outside the image reads as 0 (zero border,
 * reading of the patch border). */
static float texel(const void* map, int dtype, int W, int H, int x, int y) {
  if (x < 0 || y < 0 || x >= W || y >= H) return 0.0f;
  size_t i = (size_t)y * (size_t)W + (size_t)x;
  if (dtype == 1) return fdo_half_to_float(((const uint16_t*)map)[i]);
  return ((const float*)map)[i];
}

static const void* view_map(const void* maps, int dtype, int W, int H, int v) {
  size_t off = (size_t)v * (size_t)W * (size_t)H * (dtype == 1 ? 2u : 4u);
  return (const char*)maps + off;
}

/* ------------------------------------------------------------------------ */
/* projection, eligibility and the Eq. (4) ranking (binary64)                */
/*
 * The calibrated pinhole camera of Sec. 3.1 maps a world point p to
 * X_c = R p + t and to the pixel u = (f_x X/Z + c_x, f_y Y/Z + c_y).
 * Everything here is evaluated in binary64 from the binary32 inputs (which
 * convert exactly), so every discrete choice below (in front, inside the
 * image, visible, confidence above zero, the ranking) is the exact
 * mathematical choice up to binary64 rounding:
 *   eligible-front  : Z > z_near
 *   eligible-inside : 0 <= u_x <= W-1 and 0 <= u_y <= H-1
 *   eligible        : front, inside and the bilinear centre confidence > 0
 *   with depth maps, also visible (Sec. 3.1.1, the score V_i^v):
 *     the texel nearest to u, (floor(u_x + 1/2), floor(u_y + 1/2)), holds a
 *     rendered camera-space depth D with |Z - D| <= vis_tau
 * The pixel position u is also the centre of the fusion patch (Sec. 3.1.3:
 * the patch is taken around the projection of the point).
 */
static int project(const float* cam, const float* p, int W, int H,
                   double z_near, double u[2], double Xc[3]) {
  const float* R = cam + 4;
  const float* t = cam + 13;
  for (int r = 0; r < 3; ++r)
    Xc[r] = (double)R[3 * r] * p[0] + (double)R[3 * r + 1] * p[1] +
            (double)R[3 * r + 2] * p[2] + (double)t[r];
  if (!(Xc[2] > z_near)) return 0;
  u[0] = (double)cam[0] * (Xc[0] / Xc[2]) + (double)cam[2];
  u[1] = (double)cam[1] * (Xc[1] / Xc[2]) + (double)cam[3];
  return u[0] >= 0.0 && u[0] <= (double)(W - 1) && u[1] >= 0.0 &&
         u[1] <= (double)(H - 1);
}

/* Sec. 3.1.1 visibility: the point's camera-space depth agrees with the
 * rendered depth at the nearest texel of its projection.  Always true
 * without depth maps; a +inf (nothing rendered) or NaN depth never is. */
static int visible(const fdo_params* prm, int v, const double* u, double Z) {
  if (!prm->depth_maps) return 1;
  const int W = prm->width, H = prm->height, dt = prm->map_dtype;
  int ix = (int)floor(u[0] + 0.5), iy = (int)floor(u[1] + 0.5);
  double D = texel(view_map(prm->depth_maps, dt, W, H, v), dt, W, H, ix, iy);
  return fabs(Z - D) <= prm->vis_tau;
}

/* Plain bilinear interpolation of a confidence map at (x, y); texels outside
 * the image read 0. */
static double bilinear_conf(const void* cmap, int dtype, int W, int H, double x,
                            double y) {
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  int ix = (int)x0, iy = (int)y0;
  return (1.0 - fx) * (1.0 - fy) * texel(cmap, dtype, W, H, ix, iy) +
         fx * (1.0 - fy) * texel(cmap, dtype, W, H, ix + 1, iy) +
         (1.0 - fx) * fy * texel(cmap, dtype, W, H, ix, iy + 1) +
         fx * fy * texel(cmap, dtype, W, H, ix + 1, iy + 1);
}

/* Eq. (4): the K eligible views with the largest centre confidence; equal
 * confidences go to the lower view index. */
int fdo_select_views(const float* p, const float* cams, int32_t n_views,
                     const void* conf_maps, const fdo_params* prm,
                     int32_t* views_out, double* u_out) {
  const int W = prm->width, H = prm->height, dt = prm->map_dtype;
  int K = prm->top_k;
  if (K > FDO_MAX_K) K = FDO_MAX_K;
  int kept = 0;
  int ids[FDO_MAX_K];
  double sc[FDO_MAX_K], us[FDO_MAX_K][2];
  for (int v = 0; v < n_views; ++v) {
    double u[2], Xc[3];
    if (!project(cams + 16 * v, p, W, H, prm->z_near, u, Xc)) continue;
    if (!visible(prm, v, u, Xc[2])) continue;
    double s = bilinear_conf(view_map(conf_maps, dt, W, H, v), dt, W, H, u[0], u[1]);
    if (!(s > 0.0)) continue;
    /* insertion into a descending list; a later view must be strictly
       better to move ahead of an earlier one */
    int pos = kept;
    while (pos > 0 && s > sc[pos - 1]) --pos;
    if (pos >= K) continue;
    int last = kept < K ? kept : K - 1;
    for (int j = last; j > pos; --j) {
      sc[j] = sc[j - 1];
      ids[j] = ids[j - 1];
      us[j][0] = us[j - 1][0];
      us[j][1] = us[j - 1][1];
    }
    sc[pos] = s;
    ids[pos] = v;
    us[pos][0] = u[0];
    us[pos][1] = u[1];
    if (kept < K) ++kept;
  }
  for (int j = 0; j < kept; ++j) {
    views_out[j] = ids[j];
    if (u_out) {
      u_out[2 * j] = us[j][0];
      u_out[2 * j + 1] = us[j][1];
    }
  }
  return kept;
}

/* ------------------------------------------------------------------------ */
/* sampler (binary64)                                                        */
/*
 * Orientation is axial (theta and theta + pi are the same line), so the
 * bilinear sample interpolates the doubled-angle vector (cos 2theta,
 * sin 2theta), each texel weighted by its bilinear weight times its
 * confidence (a background texel, C = 0, is no measurement).  Confidence is
 * interpolated plainly.  A zero doubled-angle sum carries no orientation.
 */
void fdo_sample(const void* theta_map, const void* conf_map, int32_t dtype,
                int32_t W, int32_t H, double x, double y, double out[3]) {
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  int ix = (int)x0, iy = (int)y0;
  double cbar = 0.0, mx = 0.0, my = 0.0;
  for (int j = 0; j < 2; ++j) {
    for (int i = 0; i < 2; ++i) {
      double w = (i ? fx : 1.0 - fx) * (j ? fy : 1.0 - fy);
      double th = texel(theta_map, dtype, W, H, ix + i, iy + j);
      double c = texel(conf_map, dtype, W, H, ix + i, iy + j);
      cbar += w * c;
      mx += w * c * cos(2.0 * th);
      my += w * c * sin(2.0 * th);
    }
  }
  double norm = hypot(mx, my);
  out[0] = cbar;
  if (norm > 0.0) {
    out[1] = 0.5 * atan2(my, mx);
    out[2] = 1.0;
  } else {
    out[1] = 0.0;
    out[2] = 0.0;
  }
}

/* ------------------------------------------------------------------------ */
/* per-point state and the objective                                         */

typedef struct {
  int k_eff;
  int views[FDO_MAX_K];
  double u[FDO_MAX_K][2];    /* projection of the point (patch centre) */
  double Xc[FDO_MAX_K][3];   /* camera-space point, binary64 */
  double R[FDO_MAX_K][9];
  double f[FDO_MAX_K][2];
  int n_samp;                /* P*P */
  double cbar[FDO_MAX_K][FDO_MAX_P * FDO_MAX_P];
  double tbar[FDO_MAX_K][FDO_MAX_P * FDO_MAX_P];
  int valid[FDO_MAX_K][FDO_MAX_P * FDO_MAX_P];
} point_state;

/* Views of Eq. (4), then the P x P patch of Sec. 3.1.3 around the projected
 * point in every selected view: offsets (a, b) in {-h..h}^2 pixels from the
 * sub-pixel centre u, each sampled bilinearly. */
static void point_setup(const float* p, const float* cams, int n_views,
                        const void* theta_maps, const void* conf_maps,
                        const fdo_params* prm, point_state* st) {
  const int W = prm->width, H = prm->height, dt = prm->map_dtype;
  const int P = prm->patch, h = (P - 1) / 2;
  double u[2 * FDO_MAX_K];
  st->k_eff = fdo_select_views(p, cams, n_views, conf_maps, prm, st->views, u);
  st->n_samp = P * P;
  for (int k = 0; k < st->k_eff; ++k) {
    const float* cam = cams + 16 * st->views[k];
    st->u[k][0] = u[2 * k];
    st->u[k][1] = u[2 * k + 1];
    for (int i = 0; i < 9; ++i) st->R[k][i] = cam[4 + i];
    st->f[k][0] = cam[0];
    st->f[k][1] = cam[1];
    for (int r = 0; r < 3; ++r)
      st->Xc[k][r] = st->R[k][3 * r] * p[0] + st->R[k][3 * r + 1] * p[1] +
                     st->R[k][3 * r + 2] * p[2] + (double)cam[13 + r];
    const void* tm = view_map(theta_maps, dt, W, H, st->views[k]);
    const void* cm = view_map(conf_maps, dt, W, H, st->views[k]);
    int s = 0;
    for (int b = -h; b <= h; ++b) {
      for (int a = -h; a <= h; ++a, ++s) {
        double o[3];
        fdo_sample(tm, cm, dt, W, H, u[2 * k] + a, u[2 * k + 1] + b, o);
        st->cbar[k][s] = o[0];
        st->tbar[k][s] = o[1];
        st->valid[k][s] = (int)o[2];
      }
    }
  }
}

/* J(d) = 1 - (1/K_eff) sum_v max_p C_p |cos(phi_v(d) - theta_p)|.
 *
 * Eq. (8): the reprojected offset of a candidate; as the offset point tends
 * to p the image offset becomes parallel to the projection Jacobian times d,
 * r_v ~ (fx (dc_x Z - X dc_z), fy (dc_y Z - Y dc_z)) with dc = R d, and a
 * perspective map sends a 3D line to a 2D line, so every finite offset along
 * d has the same image direction.  Eq. (9): bidirectional similarity of unit
 * r_v and the unit map orientation, |cos(phi - theta)|.  Eq. (10): times the
 * patch confidence.  Eq. (11): maximum over the patch (the text's "maximal
 * matching response").  Views are combined by their mean; J is one minus
 * that mean so that the best direction minimises J. */
static double objective(const point_state* st, const double* d) {
  if (st->k_eff == 0) return INFINITY;
  double sum = 0.0;
  for (int k = 0; k < st->k_eff; ++k) {
    const double* R = st->R[k];
    double dc[3];
    for (int r = 0; r < 3; ++r)
      dc[r] = R[3 * r] * d[0] + R[3 * r + 1] * d[1] + R[3 * r + 2] * d[2];
    const double X = st->Xc[k][0], Y = st->Xc[k][1], Z = st->Xc[k][2];
    double rx = st->f[k][0] * (dc[0] * Z - X * dc[2]);
    double ry = st->f[k][1] * (dc[1] * Z - Y * dc[2]);
    double best = 0.0;
    if (rx != 0.0 || ry != 0.0) {
      double phi = atan2(ry, rx);
      for (int s = 0; s < st->n_samp; ++s) {
        if (!st->valid[k][s]) continue;
        double L = st->cbar[k][s] * fabs(cos(phi - st->tbar[k][s]));
        if (L > best) best = L;
      }
    }
    sum += best;
  }
  return 1.0 - sum / (double)st->k_eff;
}

double fdo_objective(const float* p, const double* d, const float* cams,
                     int32_t n_views, const void* theta_maps,
                     const void* conf_maps, const fdo_params* prm) {
  point_state* st = (point_state*)malloc(sizeof(point_state));
  point_setup(p, cams, n_views, theta_maps, conf_maps, prm, st);
  double J = objective(st, d);
  free(st);
  return J;
}

int fdo_objective_many(const float* p, const double* dirs, int64_t m,
                       const float* cams, int32_t n_views,
                       const void* theta_maps, const void* conf_maps,
                       const fdo_params* prm, double* J_out,
                       int32_t n_threads) {
  point_state* st = (point_state*)malloc(sizeof(point_state));
  point_setup(p, cams, n_views, theta_maps, conf_maps, prm, st);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < m; ++i) J_out[i] = objective(st, dirs + 3 * i);
  free(st);
  return 0;
}

int fdo_objective_each(const float* points, const double* dirs, int64_t n,
                       const float* cams, int32_t n_views,
                       const void* theta_maps, const void* conf_maps,
                       const fdo_params* prm, double* J_out, int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    point_state* st = (point_state*)malloc(sizeof(point_state));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
      point_setup(points + 3 * i, cams, n_views, theta_maps, conf_maps, prm, st);
      J_out[i] = objective(st, dirs + 3 * i);
    }
    free(st);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* candidate search                                                          */

/* Hemisphere Fibonacci lattice (Gonzalez 2010, restricted to z > 0, which
 * covers every axial direction once since d and -d are the same line):
 * z_k = 1 - (k + 1/2)/n, rho = sqrt(1 - z^2), psi_k = k pi (3 - sqrt 5). */
void fdo_lattice(int32_t n, double* dirs) {
  const double golden = FDO_PI * (3.0 - sqrt(5.0));
  for (int k = 0; k < n; ++k) {
    double z = 1.0 - (k + 0.5) / (double)n;
    double rho = sqrt(fmax(0.0, 1.0 - z * z));
    double psi = golden * (double)k;
    dirs[3 * k] = rho * cos(psi);
    dirs[3 * k + 1] = rho * sin(psi);
    dirs[3 * k + 2] = z;
  }
}

/* Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin, "Building an
 * Orthonormal Basis, Revisited", JCGT 6(1), 2017. */
void fdo_onb(const double* n, double* e1, double* e2) {
  double sign = copysign(1.0, n[2]);
  double a = -1.0 / (sign + n[2]);
  double b = n[0] * n[1] * a;
  e1[0] = 1.0 + sign * n[0] * n[0] * a;
  e1[1] = sign * b;
  e1[2] = -sign * n[0];
  e2[0] = b;
  e2[1] = sign + n[1] * n[1] * a;
  e2[2] = -n[1];
}

static void normalize3(double* v) {
  double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= l;
  v[1] /= l;
  v[2] /= l;
}

static double default_step0(int n_candidates) {
  return 0.5 * sqrt(2.0 * FDO_PI / (double)n_candidates);
}

/* Pattern search: each iteration tries the six directions at angle alpha
 * around d (stencil angles j pi/3 in the basis of fdo_onb); the best of them
 * (lowest index among equals) replaces d only if strictly better; alpha then
 * halves.  trace (optional) receives J after every iteration. */
static void refine(const point_state* st, double* d, double* Jd, int iters,
                   double alpha, double* trace) {
  for (int t = 0; t < iters; ++t) {
    double e1[3], e2[3];
    fdo_onb(d, e1, e2);
    double ca = cos(alpha), sa = sin(alpha);
    int best = -1;
    double Jbest = 0.0, cbest[3] = {0, 0, 0};
    for (int j = 0; j < 6; ++j) {
      double cj = cos(j * FDO_PI / 3.0), sj = sin(j * FDO_PI / 3.0);
      double c[3];
      for (int r = 0; r < 3; ++r)
        c[r] = ca * d[r] + sa * (cj * e1[r] + sj * e2[r]);
      normalize3(c);
      double J = objective(st, c);
      if (best < 0 || J < Jbest) {
        best = j;
        Jbest = J;
        cbest[0] = c[0];
        cbest[1] = c[1];
        cbest[2] = c[2];
      }
    }
    if (Jbest < *Jd) {
      d[0] = cbest[0];
      d[1] = cbest[1];
      d[2] = cbest[2];
      *Jd = Jbest;
    }
    if (trace) trace[t] = *Jd;
    alpha *= 0.5;
  }
}

/* d and -d are the same strand line; report the representative with z > 0,
 * else y > 0, else x >= 0. */
static void canonical_sign(double* d) {
  int flip;
  if (d[2] != 0.0)
    flip = d[2] < 0.0;
  else if (d[1] != 0.0)
    flip = d[1] < 0.0;
  else
    flip = d[0] < 0.0;
  if (flip) {
    d[0] = -d[0];
    d[1] = -d[1];
    d[2] = -d[2];
  }
}

/* Eq. (12): the candidate with the best patch consistency (lowest J; the
 * first of equal values), then the pattern-search refinement. */
static void fuse_point(const point_state* st, const fdo_params* prm,
                       const double* lattice, double* dir, double* cost,
                       double* trace, int* lattice_best) {
  if (st->k_eff == 0) {
    dir[0] = dir[1] = dir[2] = 0.0;
    *cost = INFINITY;
    if (lattice_best) *lattice_best = -1;
    return;
  }
  int best = 0;
  double Jbest = objective(st, lattice);
  for (int k = 1; k < prm->n_candidates; ++k) {
    double J = objective(st, lattice + 3 * k);
    if (J < Jbest) {
      Jbest = J;
      best = k;
    }
  }
  double d[3] = {lattice[3 * best], lattice[3 * best + 1],
                 lattice[3 * best + 2]};
  if (trace) trace[0] = Jbest;
  if (lattice_best) *lattice_best = best;
  double a0 = prm->refine_step0 > 0.0 ? prm->refine_step0
                                      : default_step0(prm->n_candidates);
  refine(st, d, &Jbest, prm->refine_iters, a0, trace ? trace + 1 : NULL);
  canonical_sign(d);
  dir[0] = d[0];
  dir[1] = d[1];
  dir[2] = d[2];
  *cost = Jbest;
}

int fdo_fuse_directions(const float* points, int64_t n_points,
                        const float* cams, int32_t n_views,
                        const void* theta_maps, const void* conf_maps,
                        const fdo_params* prm, double* dirs, double* costs,
                        int32_t n_threads) {
  double* lattice = (double*)malloc(sizeof(double) * 3 * prm->n_candidates);
  fdo_lattice(prm->n_candidates, lattice);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    point_state* st = (point_state*)malloc(sizeof(point_state));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n_points; ++i) {
      point_setup(points + 3 * i, cams, n_views, theta_maps, conf_maps, prm,
                  st);
      fuse_point(st, prm, lattice, dirs + 3 * i, costs + i, NULL, NULL);
    }
    free(st);
  }
  free(lattice);
  return 0;
}

int fdo_fuse_trace(const float* p, const float* cams, int32_t n_views,
                   const void* theta_maps, const void* conf_maps,
                   const fdo_params* prm, double* dir, double* trace,
                   int32_t* lattice_best) {
  double* lattice = (double*)malloc(sizeof(double) * 3 * prm->n_candidates);
  fdo_lattice(prm->n_candidates, lattice);
  point_state* st = (point_state*)malloc(sizeof(point_state));
  point_setup(p, cams, n_views, theta_maps, conf_maps, prm, st);
  double cost;
  int lb = -1;
  fuse_point(st, prm, lattice, dir, &cost, trace, &lb);
  if (lattice_best) *lattice_best = lb;
  int k = st->k_eff;
  free(st);
  free(lattice);
  return k;
}

int fdo_fuse_learned(const float* points, int64_t n_points, const float* cams,
                     int32_t n_views, const void* theta_maps,
                     const void* conf_maps, const fdo_params* prm,
                     const double* proposals, int32_t learned_iters,
                     double learned_step0, double tau, double* dirs,
                     double* costs, int32_t* fell_back, int32_t n_threads) {
  double* lattice = (double*)malloc(sizeof(double) * 3 * prm->n_candidates);
  fdo_lattice(prm->n_candidates, lattice);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    point_state* st = (point_state*)malloc(sizeof(point_state));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n_points; ++i) {
      point_setup(points + 3 * i, cams, n_views, theta_maps, conf_maps, prm,
                  st);
      const double* q = proposals + 3 * i;
      double l = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      int ok = st->k_eff > 0 && isfinite(l) && l > 0.0;
      double d[3] = {0, 0, 0}, J = INFINITY;
      if (ok) {
        d[0] = q[0] / l;
        d[1] = q[1] / l;
        d[2] = q[2] / l;
        J = objective(st, d);
        refine(st, d, &J, learned_iters, learned_step0, NULL);
        ok = J <= tau;
      }
      if (ok) {
        canonical_sign(d);
        dirs[3 * i] = d[0];
        dirs[3 * i + 1] = d[1];
        dirs[3 * i + 2] = d[2];
        costs[i] = J;
        fell_back[i] = 0;
      } else {
        fuse_point(st, prm, lattice, dirs + 3 * i, costs + i, NULL, NULL);
        fell_back[i] = 1;
      }
    }
    free(st);
  }
  free(lattice);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* proposal-network features                                                 */
/*
 * The n_slots most frontal views among the eligible ones (project() and
 * visible() above), ranked in binary64 by the cosine between the
 * point -> camera-centre direction a = c - p (camera centre c = -R^T t) and
 * the outward direction b = p - o:
 *   score = (a . b) / |a|
 * |b| is common to every view of a point and does not change the ranking;
 * equal scores go to the lower view index.
 */
static double frontal_score(const float* cam, const float* p, const float* o) {
  const float* R = cam + 4;
  const float* t = cam + 13;
  double a[3], b[3];
  for (int k = 0; k < 3; ++k) {
    double c = -((double)R[k] * t[0] + (double)R[3 + k] * t[1] + (double)R[6 + k] * t[2]);
    a[k] = c - (double)p[k];
    b[k] = (double)p[k] - (double)o[k];
  }
  return (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) /
         sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
}

int fdo_features(const float* points, int64_t n_points, const float* cams,
                 int32_t n_views, const void* theta_maps,
                 const void* conf_maps, const fdo_params* prm,
                 const float* head_centre, int32_t n_slots, double* feats,
                 int32_t n_threads) {
  const int W = prm->width, H = prm->height, dt = prm->map_dtype;
  const int F = 7 * n_slots;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n_points; ++i) {
    const float* p = points + 3 * i;
    int ids[64];
    double sc[64], us[64][2];
    int kept = 0, S = n_slots > 64 ? 64 : n_slots;
    for (int v = 0; v < n_views; ++v) {
      double u[2], Xc[3];
      if (!project(cams + 16 * v, p, W, H, prm->z_near, u, Xc)) continue;
      if (!visible(prm, v, u, Xc[2])) continue;
      double s = frontal_score(cams + 16 * v, p, head_centre);
      int pos = kept;
      while (pos > 0 && s > sc[pos - 1]) --pos;
      if (pos >= S) continue;
      int last = kept < S ? kept : S - 1;
      for (int j = last; j > pos; --j) {
        sc[j] = sc[j - 1];
        ids[j] = ids[j - 1];
        us[j][0] = us[j - 1][0];
        us[j][1] = us[j - 1][1];
      }
      sc[pos] = s;
      ids[pos] = v;
      us[pos][0] = u[0];
      us[pos][1] = u[1];
      if (kept < S) ++kept;
    }
    double* f = feats + (size_t)i * F;
    memset(f, 0, sizeof(double) * F);
    for (int j = 0; j < kept; ++j) {
      const float* cam = cams + 16 * ids[j];
      const void* tm = view_map(theta_maps, dt, W, H, ids[j]);
      const void* cm = view_map(conf_maps, dt, W, H, ids[j]);
      /* bilinear doubled-angle vector and confidence at the projection */
      double x = us[j][0], y = us[j][1];
      double x0 = floor(x), y0 = floor(y), fx = x - x0, fy = y - y0;
      double cbar = 0, mx = 0, my = 0;
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          double w = (a ? fx : 1 - fx) * (b ? fy : 1 - fy);
          double th = texel(tm, dt, W, H, (int)x0 + a, (int)y0 + b);
          double c = texel(cm, dt, W, H, (int)x0 + a, (int)y0 + b);
          cbar += w * c;
          mx += w * c * cos(2 * th);
          my += w * c * sin(2 * th);
        }
      /* unit point -> camera-centre direction, c = -R^T t */
      double R[9], t[3], c[3], v[3];
      for (int k = 0; k < 9; ++k) R[k] = cam[4 + k];
      for (int k = 0; k < 3; ++k) t[k] = cam[13 + k];
      for (int k = 0; k < 3; ++k)
        c[k] = -(R[k] * t[0] + R[3 + k] * t[1] + R[6 + k] * t[2]);
      for (int k = 0; k < 3; ++k) v[k] = c[k] - (double)p[k];
      normalize3(v);
      /* The observed image line through the projection back-projects to a
       * plane through the camera centre that contains the line of sight v.
       * Its direction across the line of sight, t = n x v (n the plane
       * normal), is expressed by its angle psi in the frame
       * e1 = normalize(z x v) (x instead of z if v is vertical), e2 = v x e1
       * perpendicular to v, so the input does not depend on the camera's
       * roll or on where the point falls in the image; the doubled angle is
       * carried with the sample's magnitude |m|. */
      double mag = hypot(mx, my);
      double qx = 0.0, qy = 0.0;
      if (mag > 0.0) {
        double th = 0.5 * atan2(my, mx);
        double Xc[3];
        for (int r = 0; r < 3; ++r)
          Xc[r] = R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2] + t[r];
        double dl[3] = {cos(th) / cam[0], sin(th) / cam[1], 0.0};
        double nc[3] = {Xc[1] * dl[2] - Xc[2] * dl[1], Xc[2] * dl[0] - Xc[0] * dl[2],
                        Xc[0] * dl[1] - Xc[1] * dl[0]};
        double nw[3];
        for (int k = 0; k < 3; ++k) nw[k] = R[k] * nc[0] + R[3 + k] * nc[1] + R[6 + k] * nc[2];
        double tt[3] = {nw[1] * v[2] - nw[2] * v[1], nw[2] * v[0] - nw[0] * v[2],
                        nw[0] * v[1] - nw[1] * v[0]};
        double up[3] = {0.0, 0.0, 1.0};
        if (fabs(v[2]) > 1.0 - 1e-9) {
          up[0] = 1.0;
          up[2] = 0.0;
        }
        double e1[3] = {up[1] * v[2] - up[2] * v[1], up[2] * v[0] - up[0] * v[2],
                        up[0] * v[1] - up[1] * v[0]};
        normalize3(e1);
        double e2[3] = {v[1] * e1[2] - v[2] * e1[1], v[2] * e1[0] - v[0] * e1[2],
                        v[0] * e1[1] - v[1] * e1[0]};
        double psi = atan2(tt[0] * e2[0] + tt[1] * e2[1] + tt[2] * e2[2],
                           tt[0] * e1[0] + tt[1] * e1[1] + tt[2] * e1[2]);
        qx = mag * cos(2.0 * psi);
        qy = mag * sin(2.0 * psi);
      }
      mx = qx;
      my = qy;
      f[7 * j + 0] = mx;
      f[7 * j + 1] = my;
      f[7 * j + 2] = cbar;
      f[7 * j + 3] = v[0];
      f[7 * j + 4] = v[1];
      f[7 * j + 5] = v[2];
      f[7 * j + 6] = 1.0;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Paper-literal candidates: multi-view direction sampling (Sec. 3.1.1,
 * Eqs. 1-3) and medoid-based direction fusion (Sec. 3.1.2, Eqs. 4-7), scored
 * by the patch consistency of Eqs. 8-12 (the objective above).
 *
 * For each view v of Eq. (4) (the visibility test needs prm->depth_maps):
 *   O_v(u)   unit image orientation (cos t, sin t), t the bilinear
 *            confidence-weighted doubled-angle mean at the projection u
 *            (the patch's centre sample); none -> the view gives no
 *            candidates
 *   Eq. (1)  u' = u + lambda O_v(u)               (pixels)
 *   Eq. (2)  z = D_v(nearest texel of u'), z_s = z + delta_s,
 *            delta_s = -Delta + 2 Delta (s - 1)/(S - 1)  (0 when S = 1);
 *            u' outside the image or z not finite -> no candidates
 *   Eq. (3)  p_s = R^T (((u'_x - c_x) z_s / f_x, (u'_y - c_y) z_s / f_y, z_s) - t)
 *   d_{v,s}  = (p_s - p) / |p_s - p|   (unit; none when z_s <= 0 or p_s = p)
 * Eqs. (5)-(7), per depth layer s over the views that gave a candidate:
 *   sigma_i = sum_j w_j |<d_i, d_j>| / sum_j w_j,  w_j = bilinear centre
 *   confidence of view j; the fused candidate is the d_i of largest sigma_i
 *   (first of equals in the order of Eq. (4)).
 * Eq. (12): the fused candidate of lowest J (first of equals); no
 * refinement.  No candidate in any layer -> direction 0, cost +inf. */

typedef struct {
  double cand[FDO_MAX_K][FDO_MAX_S][3];
  int ok[FDO_MAX_K][FDO_MAX_S];
  double w[FDO_MAX_K];
  int medoid[FDO_MAX_S];     /* view slot of the fused candidate, -1 = empty */
  double fused[FDO_MAX_S][3];
  double J[FDO_MAX_S];
  int s_best;
} fpmvo_trace;

static void fpmvo_point(const point_state* st, const float* p, const float* cams,
                        const fdo_params* prm, double lambda, int S, double delta,
                        double* dir, double* cost, fpmvo_trace* tr) {
  const int W = prm->width, H = prm->height, dt = prm->map_dtype;
  const int P = prm->patch, h = (P - 1) / 2, centre = h * P + h;
  const int K = st->k_eff;
  for (int k = 0; k < K; ++k) {
    tr->w[k] = st->cbar[k][centre];
    for (int s = 0; s < S; ++s) tr->ok[k][s] = 0;
    if (!st->valid[k][centre]) continue;
    const double t = st->tbar[k][centre];
    const double ux = st->u[k][0] + lambda * cos(t), uy = st->u[k][1] + lambda * sin(t);
    if (!(ux >= 0.0 && ux <= W - 1 && uy >= 0.0 && uy <= H - 1)) continue;
    const int ix = (int)floor(ux + 0.5), iy = (int)floor(uy + 0.5);
    const double z =
        texel(view_map(prm->depth_maps, dt, W, H, st->views[k]), dt, W, H, ix, iy);
    if (!isfinite(z)) continue;
    const float* cam = cams + 16 * st->views[k];
    for (int s = 0; s < S; ++s) {
      const double zs = z + (S > 1 ? -delta + 2.0 * delta * s / (S - 1) : 0.0);
      if (!(zs > 0.0)) continue;
      const double xc[3] = {(ux - cam[2]) * zs / cam[0] - cam[13],
                            (uy - cam[3]) * zs / cam[1] - cam[14], zs - cam[15]};
      double d[3];
      for (int r = 0; r < 3; ++r)
        d[r] = st->R[k][r] * xc[0] + st->R[k][3 + r] * xc[1] +
               st->R[k][6 + r] * xc[2] - (double)p[r];
      const double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (!(n > 0.0)) continue;
      for (int r = 0; r < 3; ++r) tr->cand[k][s][r] = d[r] / n;
      tr->ok[k][s] = 1;
    }
  }
  tr->s_best = -1;
  double Jbest = INFINITY;
  for (int s = 0; s < S; ++s) {
    tr->medoid[s] = -1;
    tr->J[s] = INFINITY;
    double wsum = 0.0, best = -INFINITY;
    for (int j = 0; j < K; ++j)
      if (tr->ok[j][s]) wsum += tr->w[j];
    for (int i = 0; i < K; ++i) {
      if (!tr->ok[i][s]) continue;
      /* G_ii = |<d_i, d_i>| = 1 for a unit direction: taken exactly */
      double num = 0.0;
      for (int j = 0; j < K; ++j) {
        if (!tr->ok[j][s]) continue;
        num += j == i ? tr->w[j]
                      : tr->w[j] * fabs(tr->cand[i][s][0] * tr->cand[j][s][0] +
                                        tr->cand[i][s][1] * tr->cand[j][s][1] +
                                        tr->cand[i][s][2] * tr->cand[j][s][2]);
      }
      const double sigma = num / wsum;
      if (sigma > best) {
        best = sigma;
        tr->medoid[s] = i;
      }
    }
    if (tr->medoid[s] < 0) continue;
    for (int r = 0; r < 3; ++r) tr->fused[s][r] = tr->cand[tr->medoid[s]][s][r];
    tr->J[s] = objective(st, tr->fused[s]);
    if (tr->J[s] < Jbest) {
      Jbest = tr->J[s];
      tr->s_best = s;
    }
  }
  if (tr->s_best < 0) {
    dir[0] = dir[1] = dir[2] = 0.0;
    *cost = INFINITY;
    return;
  }
  double d[3] = {tr->fused[tr->s_best][0], tr->fused[tr->s_best][1],
                 tr->fused[tr->s_best][2]};
  canonical_sign(d);
  dir[0] = d[0];
  dir[1] = d[1];
  dir[2] = d[2];
  *cost = Jbest;
}

int fdo_fpmvo(const float* points, int64_t n_points, const float* cams,
              int32_t n_views, const void* theta_maps, const void* conf_maps,
              const fdo_params* prm, double lambda, int32_t n_samples,
              double delta, double* dirs, double* costs, int32_t n_threads) {
  if (!prm->depth_maps || n_samples < 1 || n_samples > FDO_MAX_S) return -1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    point_state* st = (point_state*)malloc(sizeof(point_state));
    fpmvo_trace* tr = (fpmvo_trace*)malloc(sizeof(fpmvo_trace));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n_points; ++i) {
      point_setup(points + 3 * i, cams, n_views, theta_maps, conf_maps, prm, st);
      fpmvo_point(st, points + 3 * i, cams, prm, lambda, n_samples, delta,
                  dirs + 3 * i, costs + i, tr);
    }
    free(tr);
    free(st);
  }
  return 0;
}

int fdo_fpmvo_trace(const float* p, const float* cams, int32_t n_views,
                    const void* theta_maps, const void* conf_maps,
                    const fdo_params* prm, double lambda, int32_t n_samples,
                    double delta, int32_t* views, double* cand, int32_t* ok,
                    double* w, int32_t* medoid, double* fused, double* J,
                    int32_t* s_best, double* dir, double* cost) {
  if (!prm->depth_maps || n_samples < 1 || n_samples > FDO_MAX_S) return -1;
  point_state* st = (point_state*)malloc(sizeof(point_state));
  fpmvo_trace* tr = (fpmvo_trace*)malloc(sizeof(fpmvo_trace));
  point_setup(p, cams, n_views, theta_maps, conf_maps, prm, st);
  fpmvo_point(st, p, cams, prm, lambda, n_samples, delta, dir, cost, tr);
  const int K = st->k_eff, S = n_samples;
  for (int k = 0; k < K; ++k) {
    views[k] = st->views[k];
    w[k] = tr->w[k];
    for (int s = 0; s < S; ++s) {
      ok[k * S + s] = tr->ok[k][s];
      for (int r = 0; r < 3; ++r)
        cand[(k * S + s) * 3 + r] = tr->ok[k][s] ? tr->cand[k][s][r] : 0.0;
    }
  }
  for (int s = 0; s < S; ++s) {
    medoid[s] = tr->medoid[s];
    J[s] = tr->J[s];
    for (int r = 0; r < 3; ++r) fused[3 * s + r] = tr->medoid[s] >= 0 ? tr->fused[s][r] : 0.0;
  }
  *s_best = tr->s_best;
  free(tr);
  free(st);
  return K;
}
