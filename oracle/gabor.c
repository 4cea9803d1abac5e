/*
 * gabor.c -- CPU oracle for 2D orientation and confidence extraction.
 *
 * TEST INFRASTRUCTURE ONLY (see fdo.h).  Plain binary64 statement of the
 * map extraction that feeds the direction search: the paper extracts its
 * orientation maps O and confidence maps C with Gabor filters (Sec. 3.1,
 * opening paragraph) and gives no filter parameters.  The readings, written
 * out here and in the design notes:
 *
 *   bank    n_orient even (cosine) Gabor kernels of radius r, orientation
 *           theta_i = i pi / n_orient (the strand direction, from image +x
 *           towards +y, like the maps), i = 0..n_orient-1.  For an offset
 *           (dx, dy): a = dx cos t + dy sin t (along the strand),
 *           b = -dx sin t + dy cos t (across it),
 *             g(dx, dy) = exp(-a^2 / (2 s_a^2) - b^2 / (2 s_b^2)) cos(2 pi b / lambda),
 *           then its mean over the (2r+1)^2 window is subtracted, so a
 *           constant image answers 0 (the carrier oscillates across the
 *           strand; a thin bright line along t answers most).
 *   response F_i(x, y) = | sum_{dx,dy} g_i(dx, dy) I(x + dx, y + dy) |, the
 *           image read as 0 outside.
 *   orientation  theta(x, y) = theta_{i*}, i* = argmax_i F_i (first of
 *           equals).
 *   confidence   w = sqrt(sum_i d(theta_i, theta)^2 (F_i - F_{i*})^2), d the
 *           angular distance between lines (min(|t - t'|, pi - |t - t'|)):
 *           large when the response is peaked around its maximum (Paris et
 *           al. 2004).  C = w / max over the image of w (0 if that is 0),
 *           so C is in [0, 1].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GB_PI 3.14159265358979323846

/* bank: n_orient x (2r+1) x (2r+1), row-major (dy major, then dx) */
void fdo_gabor_bank(int32_t n_orient, int32_t radius, double sigma_along,
                    double sigma_across, double wavelength, double* bank) {
  const int w = 2 * radius + 1;
  for (int i = 0; i < n_orient; ++i) {
    const double t = GB_PI * i / n_orient, ct = cos(t), st = sin(t);
    double* g = bank + (size_t)i * w * w;
    double mean = 0.0;
    for (int dy = -radius; dy <= radius; ++dy)
      for (int dx = -radius; dx <= radius; ++dx) {
        const double a = dx * ct + dy * st, b = -dx * st + dy * ct;
        const double v = exp(-a * a / (2 * sigma_along * sigma_along) -
                             b * b / (2 * sigma_across * sigma_across)) *
                         cos(2 * GB_PI * b / wavelength);
        g[(dy + radius) * w + (dx + radius)] = v;
        mean += v;
      }
    mean /= (double)(w * w);
    for (int k = 0; k < w * w; ++k) g[k] -= mean;
  }
}

static double line_dist(double a, double b) {
  double d = fabs(a - b);
  return d < GB_PI - d ? d : GB_PI - d;
}

/* One image: theta_out, conf_out (H x W).  resp_out (optional): the
 * n_orient responses of every pixel, (H x W) x n_orient.  raw_out
 * (optional): w before normalisation.  Returns the normaliser max w. */
double fdo_gabor(const float* image, int32_t W, int32_t H, int32_t n_orient,
                 int32_t radius, const double* bank, double* theta_out,
                 double* conf_out, double* resp_out, double* raw_out,
                 int32_t n_threads) {
  const int w = 2 * radius + 1;
  double* raw = (double*)malloc(sizeof(double) * (size_t)W * H);
  double wmax = 0.0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
  {
    double* F = (double*)malloc(sizeof(double) * n_orient);
    double local_max = 0.0;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t p = 0; p < (int64_t)W * H; ++p) {
      const int x = (int)(p % W), y = (int)(p / W);
      for (int i = 0; i < n_orient; ++i) {
        const double* g = bank + (size_t)i * w * w;
        double s = 0.0;
        for (int dy = -radius; dy <= radius; ++dy) {
          const int yy = y + dy;
          if (yy < 0 || yy >= H) continue;
          for (int dx = -radius; dx <= radius; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= W) continue;
            s += g[(dy + radius) * w + (dx + radius)] * (double)image[(size_t)yy * W + xx];
          }
        }
        F[i] = fabs(s);
      }
      int best = 0;
      for (int i = 1; i < n_orient; ++i)
        if (F[i] > F[best]) best = i;
      const double tb = GB_PI * best / n_orient;
      double acc = 0.0;
      for (int i = 0; i < n_orient; ++i) {
        const double d = line_dist(GB_PI * i / n_orient, tb), e = F[i] - F[best];
        acc += d * d * e * e;
      }
      theta_out[p] = tb;
      raw[p] = sqrt(acc);
      if (raw[p] > local_max) local_max = raw[p];
      if (resp_out) memcpy(resp_out + (size_t)p * n_orient, F, sizeof(double) * n_orient);
    }
#ifdef _OPENMP
#pragma omp critical
#endif
    if (local_max > wmax) wmax = local_max;
    free(F);
  }
  for (int64_t p = 0; p < (int64_t)W * H; ++p) {
    conf_out[p] = wmax > 0.0 ? raw[p] / wmax : 0.0;
    if (raw_out) raw_out[p] = raw[p];
  }
  free(raw);
  return wmax;
}
