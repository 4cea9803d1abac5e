/*
 * fdo.h -- CPU oracle for fusion-patch multi-view direction optimisation.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, double-precision
 * statement of what the direction-fusion path computes.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source, header, table or helper with the GPU library, and the GPU
 * library never calls it.
 *
 * Paper: "EfficientMonoHair: Fast Strand-Level Reconstruction from Monocular
 * Video via Multi-View Direction Fusion", Sec. 3.1 (FPMVO), in particular
 * Eq. (4) (top-K confident views), Eq. (8) (reprojected candidate offset),
 * Eqs. (9)-(11) (bidirectional, confidence-weighted, patch-max consistency) and
 * Eq. (12) (best candidate).  Where the paper is silent the readings are listed
 * in the design notes of the repository; each function below names the one it
 * takes.
 *
 * Camera record: 16 binary32 values  fx, fy, cx, cy, R[9] (row-major,
 * world->camera), t[3]; a world point p maps to X_c = R p + t (x right,
 * y down, z forward) and to pixel (fx X/Z + cx, fy Y/Z + cy); texel (i, j)
 * is centred on pixel coordinate (i, j).
 *
 * Maps: V x H x W row-major; orientation theta in [0, pi] radians measured
 * from image +x towards +y, confidence C in [0, 1].  map_dtype 0 = binary32,
 * 1 = binary16.
 *
 * Parity status: every function here is pinned by the CPU test suite (closed
 * forms, brute force, invariances, finite differences) except where its
 * comment says "parity unpinned".
 */
#ifndef FDO_H
#define FDO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdo_params {
  int32_t width, height;
  int32_t map_dtype;    /* 0 = f32, 1 = f16 */
  int32_t patch;        /* P, odd, 1..7 */
  int32_t n_candidates; /* hemisphere lattice size */
  int32_t refine_iters; /* pattern-search iterations */
  double refine_step0;  /* first stencil angle in radians; <= 0 -> 0.5*sqrt(2*pi/n_candidates) */
  int32_t top_k;        /* K of Eq. (4) */
  double z_near;        /* eligibility: camera-space Z > z_near */
  /* Optional visibility test of Sec. 3.1.1 (the score V_i^v): when
   * depth_maps is not NULL (V x H x W, camera-space Z in the map dtype,
   * +inf where nothing was rendered) a view is eligible only if
   * |Z - D_v(nearest texel of u)| <= vis_tau. */
  const void* depth_maps;
  double vis_tau;
} fdo_params;

/* binary16 -> binary32, exact. */
float fdo_half_to_float(uint16_t h);

/* Eq. (4) view selection for one point, in binary64: eligible views (in
 * front, projecting inside the image, positive bilinear centre confidence
 * and, with depth maps, visible) ranked by that confidence, equal values to
 * the lower view index.  Writes up to top_k view ids (best first) and their
 * pixel positions (u_out[2*k], u_out[2*k+1]; may be NULL); returns K_eff. */
int fdo_select_views(const float* p, const float* cams, int32_t n_views,
                     const void* conf_maps, const fdo_params* prm,
                     int32_t* views_out, double* u_out);

/* Bilinear, confidence-weighted doubled-angle sample at continuous pixel
 * position (x, y) of one view.  out[0] = interpolated confidence,
 * out[1] = mean orientation in [-pi/2, pi/2], out[2] = 1 if the sample carries
 * an orientation, else 0. */
void fdo_sample(const void* theta_map, const void* conf_map, int32_t dtype,
                int32_t W, int32_t H, double x, double y, double out[3]);

/* Objective J(d) of one point for a direction d (need not be unit), from
 * scratch: view selection, patch sampling, Eqs. (8)-(11), mean over views.
 * Returns +inf when no view is eligible. */
double fdo_objective(const float* p, const double* d, const float* cams,
                     int32_t n_views, const void* theta_maps,
                     const void* conf_maps, const fdo_params* prm);

/* J for many directions of one point (M x 3, row-major) into J_out[M]. */
int fdo_objective_many(const float* p, const double* dirs, int64_t m,
                       const float* cams, int32_t n_views,
                       const void* theta_maps, const void* conf_maps,
                       const fdo_params* prm, double* J_out, int32_t n_threads);

/* J of point i for its own direction dirs[i] (N x 3), i = 0..n-1. */
int fdo_objective_each(const float* points, const double* dirs, int64_t n,
                       const float* cams, int32_t n_views,
                       const void* theta_maps, const void* conf_maps,
                       const fdo_params* prm, double* J_out, int32_t n_threads);

/* Hemisphere Fibonacci lattice of n unit directions (n x 3). */
void fdo_lattice(int32_t n, double* dirs);

/* Orthonormal basis (e1, e2) of unit n (Duff et al., JCGT 2017). */
void fdo_onb(const double* n, double* e1, double* e2);

/* Plain method for all points (OpenMP over points).  dirs N x 3 (unit,
 * canonical sign) and costs N; points without an eligible view get dir 0 and
 * cost +inf.  n_threads <= 0 uses the OpenMP default.  Returns 0. */
int fdo_fuse_directions(const float* points, int64_t n_points,
                        const float* cams, int32_t n_views,
                        const void* theta_maps, const void* conf_maps,
                        const fdo_params* prm, double* dirs, double* costs,
                        int32_t n_threads);

/* One point, with the search traced: lattice_best = index of the lattice
 * argmin, trace[0] = J after the lattice, trace[1 + t] = J after refinement
 * iteration t (refine_iters + 1 values).  Returns K_eff. */
int fdo_fuse_trace(const float* p, const float* cams, int32_t n_views,
                   const void* theta_maps, const void* conf_maps,
                   const fdo_params* prm, double* dir, double* trace,
                   int32_t* lattice_best);

/* Learned form: start from a proposal direction per point (N x 3), run
 * learned_iters pattern-search iterations from step learned_step0, accept if
 * J <= tau, otherwise return the plain result.  fell_back[i] = 1 when the
 * plain result was used.  Proposals that are not finite or are zero always
 * fall back. */
int fdo_fuse_learned(const float* points, int64_t n_points, const float* cams,
                     int32_t n_views, const void* theta_maps,
                     const void* conf_maps, const fdo_params* prm,
                     const double* proposals, int32_t learned_iters,
                     double learned_step0, double tau, double* dirs,
                     double* costs, int32_t* fell_back, int32_t n_threads);

/* Proposal-network input features: the n_slots most frontal views (ranked by
 * the cosine between the point->camera direction and the outward direction
 * p - head_centre), each slot
 * (q_x, q_y, C, v_x, v_y, v_z, valid): v is the unit point->camera
 * direction, C the bilinear confidence, and (q_x, q_y) = |m| (cos 2psi,
 * sin 2psi) where m is the bilinear confidence-weighted doubled-angle vector
 * and psi the angle, in a frame perpendicular to v, of the plane that the
 * observed image orientation back-projects to (see fdo.c).
 * feats: N x (7 n_slots).  Parity unpinned against the paper (the network
 * and its inputs are not in it); pinned by geometry in the tests. */
int fdo_features(const float* points, int64_t n_points, const float* cams,
                 int32_t n_views, const void* theta_maps,
                 const void* conf_maps, const fdo_params* prm,
                 const float* head_centre, int32_t n_slots, double* feats,
                 int32_t n_threads);

/* Paper-literal candidates (Sec. 3.1.1-3.1.2, Eqs. 1-7) scored by Eq. (12):
 * per view of Eq. (4) S depth-layer candidates from the pixel offset
 * lambda O_v(u) along the observed orientation and the depth map (depth
 * samples z + delta_s across [-delta, delta]), the confidence-weighted
 * medoid of each layer, and the layer whose fused candidate has the lowest
 * J.  Needs prm->depth_maps; 1 <= n_samples <= 16.  Returns 0, or -1 on bad
 * arguments.  The readings are written out in fdo.c. */
int fdo_fpmvo(const float* points, int64_t n_points, const float* cams,
              int32_t n_views, const void* theta_maps, const void* conf_maps,
              const fdo_params* prm, double lambda, int32_t n_samples,
              double delta, double* dirs, double* costs, int32_t n_threads);

/* One point, traced: views[K], cand[K][S][3] and ok[K][S] (per view and
 * layer), w[K], medoid[S] (view slot or -1), fused[S][3], J[S], s_best, and
 * the output dir / cost.  Returns K_eff (or -1). */
int fdo_fpmvo_trace(const float* p, const float* cams, int32_t n_views,
                    const void* theta_maps, const void* conf_maps,
                    const fdo_params* prm, double lambda, int32_t n_samples,
                    double delta, int32_t* views, double* cand, int32_t* ok,
                    double* w, int32_t* medoid, double* fused, double* J,
                    int32_t* s_best, double* dir, double* cost);

/* ---- direction-proposal MLP: 112 -> 256 -> 256 -> 256 -> 3 ---------------
 * Flat parameter order: W1[112][256], b1[256], W2[256][256], b2[256],
 * W3[256][256], b3[256], W4[256][3], b4[3]  (161283 values; y = x W + b).
 * GELU is the tanh form of Hendrycks & Gimpel (2016).  Output y/|y|.
 * bf16 = 0: binary64 throughout.  bf16 = 1: weights, layer inputs and the
 * back-propagated pre-activation gradients are rounded to bfloat16
 * (round-to-nearest-even), products are exact and sums are carried in
 * binary64 then rounded to binary32 per layer, as a matrix unit with binary32
 * accumulation would produce up to summation order. */
int64_t fdo_mlp_n_params(void);
int fdo_mlp_forward(const double* params, const float* x, int32_t batch,
                    int32_t bf16, double* y_unit);
/* Mean axial loss 1 - (y_unit . target)^2 over the batch; grad (n_params)
 * receives its gradient. */
double fdo_mlp_loss_grad(const double* params, const float* x,
                         const float* targets, int32_t batch, int32_t bf16,
                         double* grad);
/* Adam (Kingma & Ba 2015), binary32 state, step counted from 1. */
void fdo_adam_step(float* w, float* m, float* v, const float* g, int64_t n,
                   int32_t step, float lr, float beta1, float beta2,
                   float eps);
/* Round-to-nearest-even binary32 -> bfloat16 -> binary32. */
float fdo_round_bf16(float x);

#ifdef __cplusplus
}
#endif
#endif
