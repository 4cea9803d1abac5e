/*
 * phg.c -- CPU oracle for parallel hair growing.
 *
 * TEST INFRASTRUCTURE ONLY (see fdo.h).  Plain statement of the two steps
 * of the paper's parallel hair growing (Sec. 3.2.1 guide-strand
 * initialisation, Sec. 3.2.2 segment growth and connection with the test of
 * Eq. 13).  The paper gives no step length, stopping rule, thresholds or
 * conflict rule; the readings, written out here and in the design notes:
 *
 *   tracing  A trace starts at its seed x_0 with a reference direction r
 *            (the seed's direction, or the volume orientation at the seed
 *            pointed away from / towards a head centre c).  Step k reads
 *            the voxel v of x_{k-1} (the volume's binary32 voxel rule) and
 *            stops if x_{k-1} is outside the grid, v is empty, its coherence
 *            is below c_min, or v had been crossed cap times or more by the
 *            strands of earlier batches (cap > 0).  The direction is the
 *            voxel orientation t, negated if t.r < 0; after the first step
 *            the trace also stops if t.r < cos(max bend).  Then
 *            x_k = x_{k-1} + s t and r = t.  At most max_steps steps.
 *            All of it in binary32 with the dot products and the step
 *            written as fused multiply-adds in a fixed order, so a trace is
 *            a deterministic function of its inputs.
 *   batches  Seeds are taken in batches of B in seed order; every strand of
 *            a batch sees the crossing counts as they were when the batch
 *            started, and after the batch each of its steps adds 1 to the
 *            count of the voxel it read (the deferred occupancy update).
 *   linking  A piece i (a traced strand or segment) may be continued by a
 *            piece j != i that accepts predecessors if
 *            |e_i - s_j| < d_max and <u_i, w_j> > cos(theta_max) (Eq. 13),
 *            e_i, u_i the end point and direction of i, s_j, w_j the start
 *            point and direction of j (both root-to-tip).  Each i proposes
 *            its nearest such j (smallest squared distance, then smallest
 *            j); each j accepts its nearest proposer (then smallest i);
 *            accepted pairs are the links.  Squared distances are
 *            binary32: dx*dx, then fma(dy, dy, .), then fma(dz, dz, .).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int64_t fdo_voxel_of(const float p[3], const float origin[3], float h, const int32_t dims[3]);

static float dot3(const float* a, const float* b) {
  return fmaf(a[2], b[2], fmaf(a[1], b[1], a[0] * b[0]));
}

/* seed_mode: 0 = seed_dirs give r; 1 = volume orientation at the seed,
 * pointed away from centre; 2 = the same pointed towards centre (a
 * backward trace).  last_dir: the direction of the last step, negated for
 * mode 2 (so it is root-to-tip along the segment); 0 without a step. */
typedef struct fdo_trace_params {
  float step;
  int32_t max_steps;
  float min_coherence;
  float max_bend_cos;
  int32_t voxel_cap;
  int32_t batch;
  int32_t seed_mode;
  float centre[3];
} fdo_trace_params;

static int trace_one(const float* x0, const float* r0, const float origin[3], float h,
                     const int32_t dims[3], const uint32_t* occ, const float* vdir,
                     const float* coh, const uint32_t* crossings, const fdo_trace_params* p,
                     float* verts, int64_t* visited, float* last_dir) {
  float x[3] = {x0[0], x0[1], x0[2]}, r[3] = {r0[0], r0[1], r0[2]};
  verts[0] = x[0];
  verts[1] = x[1];
  verts[2] = x[2];
  int n = 1;
  last_dir[0] = last_dir[1] = last_dir[2] = 0.0f;
  for (int k = 1; k <= p->max_steps; ++k) {
    const int64_t v = fdo_voxel_of(x, origin, h, dims);
    if (v < 0 || occ[v] == 0u || !(coh[v] >= p->min_coherence)) break;
    if (p->voxel_cap > 0 && crossings[v] >= (uint32_t)p->voxel_cap) break;
    float t[3] = {vdir[3 * v], vdir[3 * v + 1], vdir[3 * v + 2]};
    if (t[0] == 0.0f && t[1] == 0.0f && t[2] == 0.0f) break; /* no orientation */
    float c = dot3(t, r);
    if (c < 0.0f) {
      t[0] = -t[0];
      t[1] = -t[1];
      t[2] = -t[2];
      c = -c;
    }
    if (k > 1 && c < p->max_bend_cos) break;
    for (int a = 0; a < 3; ++a) {
      x[a] = fmaf(p->step, t[a], x[a]);
      r[a] = t[a];
      verts[3 * n + a] = x[a];
    }
    visited[n - 1] = v;
    ++n;
  }
  if (n > 1) {
    const float sg = p->seed_mode == 2 ? -1.0f : 1.0f;
    for (int a = 0; a < 3; ++a) last_dir[a] = sg * r[a];
  }
  return n;
}

/* Traces n_seeds seeds.  crossings (nv, in/out) holds the counts of earlier
 * calls and receives this call's.  verts: n_seeds x (max_steps + 1) x 3
 * (vertices past n_verts[i] are left as they are); n_verts: n_seeds (>= 1,
 * the seed itself); last_dir: n_seeds x 3.  Returns 0. */
int fdo_grow(const float origin[3], float h, const int32_t dims[3], const uint32_t* occ,
             const float* vdir, const float* coh, const float* seeds, const float* seed_dirs,
             int32_t n_seeds, const fdo_trace_params* p, uint32_t* crossings, float* verts,
             int32_t* n_verts, float* last_dir) {
  const int stride = p->max_steps + 1;
  int64_t* visited = (int64_t*)malloc(sizeof(int64_t) * (size_t)(p->max_steps > 0 ? p->max_steps : 1) *
                                      (size_t)(p->batch > 0 ? p->batch : 1));
  for (int32_t b0 = 0; b0 < n_seeds; b0 += p->batch) {
    const int32_t b1 = b0 + p->batch < n_seeds ? b0 + p->batch : n_seeds;
    for (int32_t i = b0; i < b1; ++i) {
      float r[3] = {0.0f, 0.0f, 0.0f};
      const float* x0 = seeds + 3 * (size_t)i;
      if (p->seed_mode == 0) {
        for (int a = 0; a < 3; ++a) r[a] = seed_dirs[3 * (size_t)i + a];
      } else {
        const int64_t v = fdo_voxel_of(x0, origin, h, dims);
        if (v >= 0) {
          float t[3] = {vdir[3 * v], vdir[3 * v + 1], vdir[3 * v + 2]};
          const float off[3] = {x0[0] - p->centre[0], x0[1] - p->centre[1], x0[2] - p->centre[2]};
          const float c = dot3(t, off);
          const int away = !(c < 0.0f);
          const float sg = (away == (p->seed_mode == 1)) ? 1.0f : -1.0f;
          for (int a = 0; a < 3; ++a) r[a] = sg * t[a];
        }
      }
      n_verts[i] = trace_one(x0, r, origin, h, dims, occ, vdir, coh, crossings, p,
                             verts + (size_t)i * stride * 3,
                             visited + (size_t)(i - b0) * (p->max_steps > 0 ? p->max_steps : 1),
                             last_dir + 3 * (size_t)i);
    }
    /* the deferred update: every step of the batch counts once */
    for (int32_t i = b0; i < b1; ++i)
      for (int k = 0; k < n_verts[i] - 1; ++k)
        ++crossings[visited[(size_t)(i - b0) * (p->max_steps > 0 ? p->max_steps : 1) + k]];
  }
  free(visited);
  return 0;
}

static float dist2(const float* a, const float* b) {
  const float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* flags: bit 0 valid, bit 1 accepts a predecessor.  succ: n, the accepted
 * successor of each piece or -1.  Brute force over all pairs. */
void fdo_link(const float* starts, const float* start_dirs, const float* ends,
              const float* end_dirs, const uint8_t* flags, int32_t n, float max_dist,
              float min_cos, int32_t* succ, int32_t n_threads) {
  const float d2max = max_dist * max_dist;
  int32_t* prop = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  float* prop_d = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int32_t i = 0; i < n; ++i) {
    prop[i] = -1;
    prop_d[i] = 0.0f;
    if (!(flags[i] & 1)) continue;
    float best = 0.0f;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i || (flags[j] & 3) != 3) continue;
      const float d2 = dist2(ends + 3 * (size_t)i, starts + 3 * (size_t)j);
      if (!(d2 < d2max)) continue;
      if (!(dot3(end_dirs + 3 * (size_t)i, start_dirs + 3 * (size_t)j) > min_cos)) continue;
      if (prop[i] < 0 || d2 < best) { /* j ascending: the first of equals stays */
        prop[i] = j;
        best = d2;
      }
    }
    prop_d[i] = best;
  }
  /* each j keeps its nearest proposer (i ascending: the first of equals) */
  int32_t* win = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t j = 0; j < n; ++j) win[j] = -1;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t j = prop[i];
    if (j < 0) continue;
    if (win[j] < 0 || prop_d[i] < prop_d[win[j]]) win[j] = i;
  }
  for (int32_t i = 0; i < n; ++i) succ[i] = -1;
  for (int32_t j = 0; j < n; ++j)
    if (win[j] >= 0) succ[win[j]] = j;
  free(win);
  free(prop);
  free(prop_d);
}

/* Strands from linked pieces (the output of Sec. 3.2.2): strand g starts
 * with guide trace g; its successor chain (succ over the n_guide guide
 * pieces, then the n_seg segments) appends each segment root to tip: the
 * backward trace reversed without its seed, then the forward trace (seed
 * included).  A chain ends at -1 or at a guide piece.  Each trace set has
 * its own stride (max_steps + 1 of its call).  lengths: n_guide vertex
 * counts; pieces: n_guide piece counts.  With out (3 x the total),
 * the vertices are written strand after strand; returns the total. */
int64_t fdo_assemble(const float* guide_v, const int32_t* guide_n, int32_t n_guide,
                     int32_t g_stride, const float* fwd_v, const int32_t* fwd_n, int32_t f_stride,
                     const float* bwd_v, const int32_t* bwd_n, int32_t b_stride, int32_t n_seg,
                     const int32_t* succ, int64_t* lengths, int32_t* pieces, float* out) {
  int64_t total = 0;
  for (int32_t g = 0; g < n_guide; ++g) {
    int64_t len = guide_n[g];
    int32_t np = 1;
    if (out)
      memcpy(out + 3 * total, guide_v + (size_t)g * g_stride * 3,
             sizeof(float) * 3 * (size_t)guide_n[g]);
    int64_t pos = total + guide_n[g];
    int32_t j = succ[g];
    for (int32_t hop = 0; j >= n_guide && j < n_guide + n_seg && hop < n_guide + n_seg; ++hop) {
      const int32_t s = j - n_guide;
      const float* b = bwd_v + (size_t)s * b_stride * 3;
      const float* f = fwd_v + (size_t)s * f_stride * 3;
      for (int k = bwd_n[s] - 1; k >= 1; --k) {
        if (out) memcpy(out + 3 * pos, b + 3 * k, sizeof(float) * 3);
        ++pos;
      }
      if (out) memcpy(out + 3 * pos, f, sizeof(float) * 3 * (size_t)fwd_n[s]);
      pos += fwd_n[s];
      len += (bwd_n[s] - 1) + fwd_n[s];
      ++np;
      j = succ[j];
    }
    lengths[g] = len;
    pieces[g] = np;
    total += len;
  }
  return total;
}
