/*
 * mlp.c -- CPU oracle for the direction-proposal network and its optimiser.
 *
 * TEST INFRASTRUCTURE ONLY (see fdo.h).  Four fully connected layers
 * 112 -> 256 -> 256 -> 256 -> 3 with GELU (tanh form, Hendrycks & Gimpel
 * 2016) after the first three, output normalised to a unit vector, axial
 * loss 1 - (y.t)^2 (a strand direction and its negation are the same line),
 * and Adam (Kingma & Ba 2015).  Plain loops; binary64 unless the bfloat16
 * emulation switch is on.
 */
#include "fdo.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { D0 = 112, D1 = 256, D2 = 256, D3 = 256, D4 = 3 };

static const int dims[5] = {D0, D1, D2, D3, D4};

int64_t fdo_mlp_n_params(void) {
  int64_t n = 0;
  for (int l = 0; l < 4; ++l) n += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
  return n;
}

float fdo_round_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) { /* inf / nan pass through */
    if (u & 0x007fffffu) u |= 0x00400000u;
    u &= 0xffff0000u;
  } else {
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
  }
  float y;
  memcpy(&y, &u, 4);
  return y;
}

static double q(double x, int bf16) {
  return bf16 ? (double)fdo_round_bf16((float)x) : x;
}

/* per-layer rounding of an accumulated sum: binary32 in emulation mode */
static double acc_out(double x, int bf16) { return bf16 ? (double)(float)x : x; }

static double gelu(double x) {
  const double c = sqrt(2.0 / 3.14159265358979323846);
  return 0.5 * x * (1.0 + tanh(c * (x + 0.044715 * x * x * x)));
}

static double gelu_grad(double x) {
  const double c = sqrt(2.0 / 3.14159265358979323846);
  double u = c * (x + 0.044715 * x * x * x);
  double th = tanh(u);
  double du = c * (1.0 + 3.0 * 0.044715 * x * x);
  return 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th * th) * du;
}

typedef struct {
  const double* W[4];
  const double* b[4];
} layer_view;

static void split_params(const double* params, layer_view* lv) {
  const double* p = params;
  for (int l = 0; l < 4; ++l) {
    lv->W[l] = p;
    p += (size_t)dims[l] * dims[l + 1];
    lv->b[l] = p;
    p += dims[l + 1];
  }
}

/* Forward pass of one sample; keeps the layer inputs h[l] (as used by the
 * products) and the pre-activations z[l]. */
typedef struct {
  double h[4][256]; /* input of layer l */
  double z[4][256]; /* pre-activation of layer l */
  double y[3];
  double norm;
} trace_t;

static void forward_one(const layer_view* lv, const float* x, int bf16,
                        trace_t* tr) {
  for (int k = 0; k < D0; ++k) tr->h[0][k] = q((double)x[k], bf16);
  for (int l = 0; l < 4; ++l) {
    const int K = dims[l], N = dims[l + 1];
    for (int n = 0; n < N; ++n) {
      double s = 0.0;
      for (int k = 0; k < K; ++k)
        s += tr->h[l][k] * q(lv->W[l][(size_t)k * N + n], bf16);
      s = acc_out(s, bf16);
      tr->z[l][n] = acc_out(s + lv->b[l][n], bf16);
    }
    if (l < 3) {
      for (int n = 0; n < N; ++n)
        tr->h[l + 1][n] = q(acc_out(gelu(tr->z[l][n]), bf16), bf16);
    }
  }
  double nn = 0.0;
  for (int j = 0; j < 3; ++j) nn += tr->z[3][j] * tr->z[3][j];
  tr->norm = sqrt(nn);
  for (int j = 0; j < 3; ++j) tr->y[j] = tr->z[3][j] / tr->norm;
}

int fdo_mlp_forward(const double* params, const float* x, int32_t batch,
                    int32_t bf16, double* y_unit) {
  layer_view lv;
  split_params(params, &lv);
  trace_t* tr = (trace_t*)malloc(sizeof(trace_t));
  for (int b = 0; b < batch; ++b) {
    forward_one(&lv, x + (size_t)b * D0, bf16, tr);
    for (int j = 0; j < 3; ++j) y_unit[3 * b + j] = tr->y[j];
  }
  free(tr);
  return 0;
}

/* Loss L = (1/B) sum_b [1 - (y_b . t_b)^2], y_b = z4_b / |z4_b|.
 * dL/dy = -2 (y.t) t / B;  dL/dz4 = (dL/dy - y (y . dL/dy)) / |z4|;
 * dL/dW_l = h_l^T dL/dz_l,  dL/db_l = sum_b dL/dz_l,
 * dL/dh_l = dL/dz_l W_l^T,  dL/dz_{l-1} = dL/dh_l * gelu'(z_{l-1}).
 * In emulation mode dL/dz_l of the three hidden layers is rounded to
 * bfloat16 where it enters a product (the bias sums use it unrounded); the
 * output layer's gradient stays in binary32. */
double fdo_mlp_loss_grad(const double* params, const float* x,
                         const float* targets, int32_t batch, int32_t bf16,
                         double* grad) {
  layer_view lv;
  split_params(params, &lv);
  const int64_t np = fdo_mlp_n_params();
  memset(grad, 0, sizeof(double) * (size_t)np);
  double* gW[4];
  double* gb[4];
  {
    double* p = grad;
    for (int l = 0; l < 4; ++l) {
      gW[l] = p;
      p += (size_t)dims[l] * dims[l + 1];
      gb[l] = p;
      p += dims[l + 1];
    }
  }
  trace_t* tr = (trace_t*)malloc(sizeof(trace_t));
  double loss = 0.0;
  double dz[256], dzq[256], dh[256];
  for (int b = 0; b < batch; ++b) {
    forward_one(&lv, x + (size_t)b * D0, bf16, tr);
    const float* t = targets + 3 * b;
    double yt = tr->y[0] * t[0] + tr->y[1] * t[1] + tr->y[2] * t[2];
    loss += 1.0 - yt * yt;
    double dy[3], ydy = 0.0;
    for (int j = 0; j < 3; ++j) {
      dy[j] = -2.0 * yt * (double)t[j] / (double)batch;
      ydy += tr->y[j] * dy[j];
    }
    for (int j = 0; j < 3; ++j) {
      dz[j] = acc_out((dy[j] - tr->y[j] * ydy) / tr->norm, bf16);
      dzq[j] = dz[j];
    }
    for (int l = 3; l >= 0; --l) {
      const int K = dims[l], N = dims[l + 1];
      /* weight and bias gradients */
      for (int k = 0; k < K; ++k)
        for (int n = 0; n < N; ++n)
          gW[l][(size_t)k * N + n] += tr->h[l][k] * dzq[n];
      for (int n = 0; n < N; ++n) gb[l][n] += dz[n];
      if (l == 0) break;
      /* back through the weights and the activation of layer l-1 */
      for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int n = 0; n < N; ++n)
          s += dzq[n] * q(lv.W[l][(size_t)k * N + n], bf16);
        dh[k] = acc_out(s, bf16);
      }
      for (int k = 0; k < K; ++k) {
        dz[k] = acc_out(dh[k] * gelu_grad(tr->z[l - 1][k]), bf16);
        dzq[k] = q(dz[k], bf16);
      }
    }
  }
  free(tr);
  return loss / (double)batch;
}

/* m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 * w <- w - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
void fdo_adam_step(float* w, float* m, float* v, const float* g, int64_t n,
                   int32_t step, float lr, float beta1, float beta2,
                   float eps) {
  double bc1 = 1.0 - pow((double)beta1, (double)step);
  double bc2 = 1.0 - pow((double)beta2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = (float)(beta1 * (double)m[i] + (1.0 - beta1) * (double)g[i]);
    v[i] = (float)(beta2 * (double)v[i] +
                   (1.0 - beta2) * (double)g[i] * (double)g[i]);
    double mh = (double)m[i] / bc1, vh = (double)v[i] / bc2;
    w[i] = (float)((double)w[i] - lr * mh / (sqrt(vh) + eps));
  }
}
