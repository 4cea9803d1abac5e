/*
 * volume.c -- CPU oracle for the occupancy and orientation volume.
 *
 * TEST INFRASTRUCTURE ONLY (see fdo.h).  Plain binary64 statement of the
 * fusion of oriented points (the outer points with their fused directions
 * and the inner points) into one occupancy / orientation volume
 * (Sec. 3.2, opening paragraph).  The paper names the volume and gives no
 * rule; the readings, written out here and in the design notes:
 *
 *   grid    origin o, cubic voxel of edge h, dims (nx, ny, nz), voxel
 *           (ix, iy, iz) at linear index (iz * ny + iy) * nx + ix.  A point
 *           belongs to voxel i_a = floor(q_a) on each axis, with
 *           q_a = (p_a - o_a) / h evaluated in binary32 (subtraction, then
 *           IEEE division), and counts only if 0 <= q_a < dims_a on all
 *           three axes (a point on a face goes to the upper voxel).
 *   occupancy  the number of points in the voxel.
 *   orientation  strand directions are lines (d and -d alike), so they are
 *           averaged through the structure tensor T = sum_i w_i d_i d_i^T
 *           over the voxel's points (w_i >= 0, the point's weight: its
 *           reliability).  The voxel's orientation is the unit eigenvector
 *           of T's largest eigenvalue l1 (sign: z > 0, else y > 0, else
 *           x >= 0); its coherence is (l1 - l2) / l1, 1 for one direction,
 *           0 for directions spread evenly in a plane or in space.  A voxel
 *           whose tensor is 0 has orientation 0 and coherence 0.
 *
 * The eigenvectors come from the cyclic Jacobi method (Golub and Van Loan,
 * Sec. 8.5) run to machine precision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* voxel of a point, or -1 outside the grid */
int64_t fdo_voxel_of(const float p[3], const float origin[3], float h, const int32_t dims[3]) {
  int32_t ix[3];
  for (int a = 0; a < 3; ++a) {
    volatile float t = p[a] - origin[a]; /* binary32, rounded here */
    volatile float q = t / h;
    if (!(q >= 0.0f) || !(q < (float)dims[a])) return -1;
    ix[a] = (int32_t)floorf(q);
  }
  return ((int64_t)ix[2] * dims[1] + ix[1]) * dims[0] + ix[0];
}

/* Eigen-decomposition of a symmetric 3x3 matrix A (row-major, 9 values):
 * eigenvalues l[0] >= l[1] >= l[2], eigenvectors as the columns of V. */
void fdo_sym3_eigen(const double* A_in, double* l, double* V) {
  double A[3][3], Q[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A[i][j] = A_in[i * 3 + j];
      Q[i][j] = i == j;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-36 * diag || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        /* the rotation that zeroes A[p][q] (the smaller angle) */
        const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) { /* A <- A J */
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) { /* A <- J^T A */
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) { /* Q <- Q J */
          const double qkp = Q[k][p], qkq = Q[k][q];
          Q[k][p] = c * qkp - s * qkq;
          Q[k][q] = s * qkp + c * qkq;
        }
      }
  }
  int ord[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i) /* descending, stable */
    for (int j = i + 1; j < 3; ++j)
      if (A[ord[j]][ord[j]] > A[ord[i]][ord[i]]) {
        const int t = ord[i];
        ord[i] = ord[j];
        ord[j] = t;
      }
  for (int k = 0; k < 3; ++k) {
    l[k] = A[ord[k]][ord[k]];
    for (int i = 0; i < 3; ++i) V[i * 3 + k] = Q[i][ord[k]];
  }
}

static void canonical_line(double* d) {
  int flip;
  if (d[2] != 0.0)
    flip = d[2] < 0.0;
  else if (d[1] != 0.0)
    flip = d[1] < 0.0;
  else
    flip = d[0] < 0.0;
  if (flip)
    for (int a = 0; a < 3; ++a) d[a] = -d[a];
}

/* Orientation and coherence of one tensor (xx, yy, zz, xy, xz, yz). */
void fdo_tensor_orientation(const double* T6, double* dir, double* coherence) {
  const double A[9] = {T6[0], T6[3], T6[4], T6[3], T6[1], T6[5], T6[4], T6[5], T6[2]};
  int zero = 1;
  for (int k = 0; k < 6; ++k) zero &= T6[k] == 0.0;
  if (zero) {
    dir[0] = dir[1] = dir[2] = 0.0;
    *coherence = 0.0;
    return;
  }
  double l[3], V[9];
  fdo_sym3_eigen(A, l, V);
  for (int a = 0; a < 3; ++a) dir[a] = V[a * 3 + 0];
  const double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  for (int a = 0; a < 3; ++a) dir[a] /= n;
  canonical_line(dir);
  *coherence = l[0] > 0.0 ? (l[0] - l[1]) / l[0] : 0.0;
}

/* points, dirs: n x 3; weights: n or NULL (all 1).  occ: nv counts;
 * tensor: nv x 6 (xx, yy, zz, xy, xz, yz); dir_out: nv x 3; coh_out: nv.
 * Returns the number of points inside the grid. */
int64_t fdo_volume(const float* points, const float* dirs, const float* weights, int64_t n,
                   const float origin[3], float h, const int32_t dims[3], uint32_t* occ,
                   double* tensor, double* dir_out, double* coh_out, int32_t n_threads) {
  const int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
  memset(occ, 0, sizeof(uint32_t) * (size_t)nv);
  memset(tensor, 0, sizeof(double) * 6 * (size_t)nv);
  int64_t inside = 0;
  for (int64_t i = 0; i < n; ++i) { /* in point order */
    const int64_t v = fdo_voxel_of(points + 3 * i, origin, h, dims);
    if (v < 0) continue;
    ++inside;
    ++occ[v];
    const double w = weights ? (double)weights[i] : 1.0;
    const double d[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]};
    double* T = tensor + 6 * v;
    T[0] += w * d[0] * d[0];
    T[1] += w * d[1] * d[1];
    T[2] += w * d[2] * d[2];
    T[3] += w * d[0] * d[1];
    T[4] += w * d[0] * d[2];
    T[5] += w * d[1] * d[2];
  }
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t v = 0; v < nv; ++v) fdo_tensor_orientation(tensor + 6 * v, dir_out + 3 * v, coh_out + v);
  return inside;
}
