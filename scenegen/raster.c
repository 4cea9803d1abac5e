/*
 * raster.c -- z-buffered line rasteriser for the synthetic scene generator.
 *
 * Renders strand polylines into per-view orientation and depth images for
 * calibrated pinhole cameras (16-float records fx, fy, cx, cy, R[9], t[3];
 * X_c = R p + t, pixel (fx X/Z + cx, fy Y/Z + cy), texel (i, j) centred on
 * pixel coordinate (i, j)).  Each polyline segment is walked in 3D with at
 * most half a pixel between samples; every sample lands on its nearest texel
 * and wins it if it is nearer than what the texel holds.  The texel then
 * stores the angle of the segment's image, in [0, pi), measured from +x
 * towards +y, and the sample's camera-space depth.  A sphere of the given
 * radius at the origin (the scalp) pre-fills the depth buffer, so strands
 * behind the head are hidden; covered_out marks the texels a strand won and
 * strand_out (optional) holds the winning strand's index (-1: none).
 *
 * Input generation only: this file is shared by nothing but the generator.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define SG_PI 3.14159265358979323846

#ifdef _OPENMP
#include <omp.h>
#endif

static void proj(const float* cam, const double* x, double* u, double* z) {
  const float* R = cam + 4;
  const float* t = cam + 13;
  double X = R[0] * x[0] + R[1] * x[1] + R[2] * x[2] + t[0];
  double Y = R[3] * x[0] + R[4] * x[1] + R[5] * x[2] + t[1];
  double Z = R[6] * x[0] + R[7] * x[1] + R[8] * x[2] + t[2];
  *z = Z;
  u[0] = cam[0] * X / Z + cam[2];
  u[1] = cam[1] * Y / Z + cam[3];
}

int scenegen_raster(const float* verts, const int64_t* offs, int64_t n_strands,
                    const float* cams, int32_t n_views, int32_t W, int32_t H,
                    double head_radius, float* theta_out, float* depth_out,
                    uint8_t* covered_out, int32_t* strand_out, int32_t n_threads) {
  const double z_near = 1e-3;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int v = 0; v < n_views; ++v) {
    const float* cam = cams + 16 * v;
    float* th = theta_out + (size_t)v * W * H;
    float* dp = depth_out + (size_t)v * W * H;
    uint8_t* cv = covered_out + (size_t)v * W * H;
    int32_t* sd = strand_out ? strand_out + (size_t)v * W * H : NULL;
    /* camera centre c = -R^T t, for the scalp-sphere depth */
    const float* R = cam + 4;
    const float* t = cam + 13;
    double c[3];
    for (int k = 0; k < 3; ++k)
      c[k] = -(R[k] * t[0] + R[3 + k] * t[1] + R[6 + k] * t[2]);
    for (int y = 0; y < H; ++y) {
      for (int x = 0; x < W; ++x) {
        size_t i = (size_t)y * W + x;
        th[i] = 0.0f;
        dp[i] = INFINITY;
        cv[i] = 0;
        if (sd) sd[i] = -1;
        if (head_radius <= 0) continue;
        /* camera ray through the pixel, camera frame then world frame */
        double rc[3] = {(x - cam[2]) / cam[0], (y - cam[3]) / cam[1], 1.0};
        double rw[3];
        for (int k = 0; k < 3; ++k)
          rw[k] = R[k] * rc[0] + R[3 + k] * rc[1] + R[6 + k] * rc[2];
        /* |c + s rw|^2 = r^2, s = camera-space depth since rc_z = 1 */
        double a = rw[0] * rw[0] + rw[1] * rw[1] + rw[2] * rw[2];
        double b = 2 * (c[0] * rw[0] + c[1] * rw[1] + c[2] * rw[2]);
        double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2] -
                    head_radius * head_radius;
        double disc = b * b - 4 * a * cc;
        if (disc >= 0) {
          double s = (-b - sqrt(disc)) / (2 * a);
          if (s > z_near) dp[i] = (float)s;
        }
      }
    }
    for (int64_t sidx = 0; sidx < n_strands; ++sidx) {
      for (int64_t e = offs[sidx]; e + 1 < offs[sidx + 1]; ++e) {
        double a[3] = {verts[3 * e], verts[3 * e + 1], verts[3 * e + 2]};
        double b[3] = {verts[3 * e + 3], verts[3 * e + 4], verts[3 * e + 5]};
        double ua[2], ub[2], za, zb;
        proj(cam, a, ua, &za);
        proj(cam, b, ub, &zb);
        if (!(za > z_near) || !(zb > z_near)) continue;
        double du = ub[0] - ua[0], dv = ub[1] - ua[1];
        double ang = atan2(dv, du);
        if (ang < 0) ang += SG_PI;
        if (ang >= SG_PI) ang -= SG_PI;
        double len = fmax(fabs(du), fabs(dv));
        int ns = (int)ceil(len / 0.5) + 1;
        if (ns > 100000) continue;
        for (int k = 0; k < ns; ++k) {
          double s = ns > 1 ? (double)k / (ns - 1) : 0.0;
          double p[3] = {a[0] + s * (b[0] - a[0]), a[1] + s * (b[1] - a[1]),
                         a[2] + s * (b[2] - a[2])};
          double u[2], z;
          proj(cam, p, u, &z);
          if (!(u[0] > -0.5 && u[0] < W - 0.5 && u[1] > -0.5 && u[1] < H - 0.5))
            continue;
          long ix = lround(u[0]), iy = lround(u[1]);
          if (ix < 0 || iy < 0 || ix >= W || iy >= H) continue;
          size_t i = (size_t)iy * W + ix;
          if (z < dp[i]) {
            dp[i] = (float)z;
            th[i] = (float)ang;
            cv[i] = 1;
            if (sd) sd[i] = (int32_t)sidx;
          }
        }
      }
    }
  }
  return 0;
}

/* For each point, the number of views in which it is visible: in front of
 * the camera, projecting inside the image, and within tau of the depth
 * stored at the nearest texel (depth maps V x H x W, float). */
int scenegen_visible_views(const float* pts, int64_t n, const float* cams,
                           int32_t n_views, int32_t W, int32_t H,
                           const float* depth, double tau, int32_t* count,
                           int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n; ++i) {
    double p[3] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
    int c = 0;
    for (int v = 0; v < n_views; ++v) {
      double u[2], z;
      proj(cams + 16 * v, p, u, &z);
      if (!(z > 1e-3)) continue;
      if (!(u[0] >= 0 && u[0] <= W - 1 && u[1] >= 0 && u[1] <= H - 1)) continue;
      long ix = (long)floor(u[0] + 0.5), iy = (long)floor(u[1] + 0.5);
      double d = depth[(size_t)v * W * H + (size_t)iy * W + ix];
      if (fabs(z - d) <= tau) ++c;
    }
    count[i] = c;
  }
  return 0;
}
