/*
 * fusedir.h -- C ABI of libfusedir.so: fusion-patch multi-view direction
 * optimisation on AMD Instinct MI355X (gfx950).
 *
 * For every 3D hair point the library projects the point and candidate
 * tangents into calibrated views, samples each view's orientation and
 * confidence maps over a P x P patch and returns the direction with the best
 * patch-fused, confidence-weighted bidirectional agreement (EfficientMonoHair,
 * Sec. 3.1: top-K confident views, Eq. (4); reprojected candidate offset,
 * Eq. (8); bidirectional similarity, confidence weighting and patch maximum,
 * Eqs. (9)-(11); best candidate, Eq. (12)).  Candidates are a hemisphere
 * Fibonacci lattice followed by a pattern-search refinement; a learned form
 * starts from a network proposal instead and falls back to the full search.
 *
 * Conventions shared by every entry point
 *   - Camera (fd_camera, 64 bytes): fx, fy, cx, cy, R (row-major,
 *     world->camera), t;  X_c = R p + t, OpenCV axes (x right, y down,
 *     z forward), pixel u = (fx X/Z + cx, fy Y/Z + cy), texel (i, j) centred
 *     on pixel coordinate (i, j).
 *   - Maps: V x H x W row-major, orientation theta in [0, pi] radians
 *     measured from image +x towards +y, confidence C in [0, 1] (0 = no
 *     measurement); element type FD_F32 (float) or FD_F16 (IEEE binary16).
 *   - Directions: unit float3, sign-canonical (z > 0, else y > 0, else
 *     x >= 0).  Cost J in [0, 1] = 1 - mean over the selected views of the
 *     patch-max confidence-weighted |cos| agreement; a point with no eligible
 *     view gets direction (0, 0, 0) and cost +inf.  This is not an error.
 *   - Pointers named "device" are HIP device pointers owned by the caller;
 *     the library never frees them.  All computation is enqueued on
 *     params->stream (a hipStream_t; NULL = the default stream) and the call
 *     returns after enqueueing: inputs must stay valid and outputs untouched
 *     until the stream has passed the call.
 *   - Return codes: FD_OK, or an error code with a message from
 *     fd_last_error() (thread-local).  On an error detected on the host
 *     nothing is enqueued and outputs are untouched.  No C++ exception
 *     crosses this interface.
 */
#ifndef FUSEDIR_H
#define FUSEDIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FD_OK = 0,
  FD_E_INVAL = 1,        /* bad argument: null pointer, size out of range ... */
  FD_E_UNSUPPORTED = 2,  /* device is not gfx950 */
  FD_E_HIP = 3,          /* HIP runtime or launch error */
  FD_E_NOMEM = 4         /* context workspace smaller than the request */
};

enum { FD_F32 = 0, FD_F16 = 1 };
/* PLAIN: lattice search + refinement of the objective.  LEARNED: network
 * proposal, short refinement, plain search as fallback.  FPMVO: the paper's
 * own candidates (Sec. 3.1.1-3.1.2, Eqs. 1-7: pixel offset along the observed
 * orientation, depth layers, back-projection, per-layer confidence-weighted
 * medoid over the top-K views) scored by the same objective (Eq. 12); needs
 * depth_maps. */
enum { FD_MODE_PLAIN = 0, FD_MODE_LEARNED = 1, FD_MODE_FPMVO = 2 };
#define FD_MAX_FPMVO_SAMPLES 16
/* Source of the learned form's starting direction.  Only FD_PROPOSAL_MLP
 * uses the network; the others replace it for testing (GIVEN reads
 * params->proposal_dirs, NAN makes every proposal invalid). */
enum { FD_PROPOSAL_MLP = 0, FD_PROPOSAL_GIVEN = 1, FD_PROPOSAL_NAN = 2 };

#define FD_MAX_TOPK 8
#define FD_MAX_PATCH 7
#define FD_MAX_VIEWS 65535
#define FD_MAX_CANDIDATES 4096
#define FD_MAX_REFINE 32
#define FD_FEATURE_SLOTS 16
#define FD_FEATURE_DIM 112 /* 16 slots x 7 */
#define FD_MAX_BATCH_SCENES 32

typedef struct fd_camera {
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
} fd_camera;

typedef struct fd_context fd_context;
typedef struct fd_mlp fd_mlp;

/* Host struct, read during the call only.  Fill it with fd_params_init. */
typedef struct fd_params {
  int32_t width, height;   /* map size W, H (>= 1, <= 32768) */
  int32_t map_dtype;       /* FD_F32 or FD_F16 */
  int32_t patch;           /* P: odd, 1..FD_MAX_PATCH (Eqs. 9-11) */
  int32_t n_candidates;    /* hemisphere lattice size, 1..FD_MAX_CANDIDATES */
  int32_t refine_iters;    /* pattern-search iterations, 0..FD_MAX_REFINE */
  float refine_step0;      /* first stencil angle (rad); <= 0: 0.5 sqrt(2 pi / n_candidates) */
  int32_t top_k;           /* K of Eq. (4), 1..FD_MAX_TOPK */
  float z_near;            /* a view is eligible only if camera-space Z > z_near */
  int32_t mode;            /* FD_MODE_PLAIN, FD_MODE_LEARNED or FD_MODE_FPMVO */
  const fd_mlp* mlp;       /* network for FD_MODE_LEARNED with FD_PROPOSAL_MLP */
  int32_t learned_iters;   /* refinement iterations after the proposal */
  float learned_step0;     /* their first stencil angle (rad) */
  float fallback_cost;     /* tau: refined cost above tau -> full search */
  int32_t proposal;        /* FD_PROPOSAL_* */
  const float* proposal_dirs; /* device N x 3, for FD_PROPOSAL_GIVEN */
  float head_centre[3];    /* world point the frontal-view ranking is relative to */
  float vis_tau;           /* visibility tolerance (metres) on |Z - D|, finite, >= 0 */
  const void* depth_maps;  /* device n_views x H x W of map_dtype: rendered camera-space
                              depth D_v (+inf where empty), or NULL.  When set, a view is
                              eligible for a point (view selection and the proposal
                              features alike) only if the point is visible in it:
                              |Z - D_v(nearest texel of u)| <= vis_tau, decided in
                              binary32 (Sec. 3.1.1, visibility score V_i^v) */
  float fpmvo_lambda;      /* FPMVO: pixel offset along the observed orientation (Eq. 1), > 0 */
  int32_t fpmvo_samples;   /* FPMVO: depth layers S (Eq. 2), 1..FD_MAX_FPMVO_SAMPLES */
  float fpmvo_delta;       /* FPMVO: layers at z + [-delta, delta] (metres, Eq. 2), >= 0 */
  void* stream;            /* hipStream_t */
  fd_context* ctx;         /* workspace; NULL = a per-device default that grows */
} fd_params;

/* Defaults: K = 5 (Sec. 3.1.2, Eq. 4), P = 5 (Sec. 4), 128 candidates,
 * 8 refinement iterations, z_near = 1e-3, plain mode, FD_F16 maps,
 * learned_iters = 2, no depth maps, vis_tau = 5e-3 (half the 10 mm depth
 * range of Sec. 3.1.1); FPMVO: lambda = 3 px, S = 5, delta = 5e-3 (the
 * 2 Delta = 10 mm range of Eq. 2). */
void fd_params_init(fd_params* params);

/* ---- context: library-owned workspace ------------------------------------
 * create: allocates the small fixed buffers on the current device (and a
 * camera table for 1024 views).
 * reserve: grows the per-point buffers to max_points points, the camera
 * table to max_views views (for one call, or the sum over the scenes of a
 * batched call) and the scene table to max_scenes; it is the only call
 * after create that allocates.  A call through a context with more views
 * than it holds returns FD_E_NOMEM.
 * A context is bound to the device current at create and must be used from
 * one stream at a time.  destroy: frees everything (synchronises the
 * device). */
int fd_context_create(fd_context** out);
int fd_context_reserve(fd_context* ctx, int64_t max_points, int32_t max_views,
                       int32_t max_scenes);
void fd_context_destroy(fd_context* ctx);

/* ---- main entry point -----------------------------------------------------
 * points      device, n_points x 3 float (metres, world frame)
 * n_points    >= 0 (0: nothing is enqueued)
 * cams        device, n_views fd_camera
 * n_views     1..FD_MAX_VIEWS
 * orient_maps device, n_views x H x W of params->map_dtype (theta)
 * conf_maps   device, same shape and type (C)
 * params      host, see fd_params
 * dirs        device, n_points x 3 float, written
 * costs       device, n_points float, written
 * Plain mode: tiling of the points by a spatial key, Eq. (4) view selection,
 * patch sampling, lattice argmin of J, pattern-search refinement.  FPMVO
 * mode: the same tiling and view selection, then the paper's candidates and
 * medoid fusion per depth layer, the fused candidate of lowest J (no
 * refinement); a point without any candidate gets direction 0 and cost
 * +inf.  Learned
 * mode: proposal (network or test hook), refinement from it, and the plain
 * search for every point whose refined cost exceeds params->fallback_cost.
 * The learned form needs a context (params->ctx or the default one). */
int fd_fuse_directions(const float* points, int64_t n_points,
                       const fd_camera* cams, int32_t n_views,
                       const void* orient_maps, const void* conf_maps,
                       const fd_params* params, float* dirs, float* costs);

/* ---- allocation-free variant ----------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the plain
 * mode of fd_fuse_directions, same arguments and results (the same kernels),
 * with its workspace in a fixed device array that the library holds on each
 * GPU it runs on until the process ends (under 16 MiB).  It allocates
 * nothing and ignores params->ctx.  n_points above FD_NOALLOC_MAX_POINTS,
 * n_views above FD_NOALLOC_MAX_VIEWS or a mode other than FD_MODE_PLAIN
 * returns FD_E_INVAL before anything is launched.  All calls on one GPU share that array: calls that overlap on
 * one GPU (several streams or threads) race and must be serialised by the
 * caller. */
#define FD_NOALLOC_MAX_POINTS 524288
#define FD_NOALLOC_MAX_VIEWS 1024
int fd_fuse_directions_noalloc(const float* points, int64_t n_points,
                               const fd_camera* cams, int32_t n_views,
                               const void* orient_maps, const void* conf_maps,
                               const fd_params* params, float* dirs, float* costs);

/* Number of points of the last learned call on this context that took the
 * full search (reads a device counter; synchronises params->stream). */
int fd_last_fallback_count(fd_context* ctx, void* stream, int64_t* out);

/* The same points split by where their full search ran: *in_place inside
 * the refinement kernel (waves in which at least half of the points needed
 * it, on the patch registers they already held), *listed by the separate
 * fallback launch over the compacted list. */
int fd_last_fallback_split(fd_context* ctx, void* stream, int64_t* listed, int64_t* in_place);

/* ---- many scenes in one launch --------------------------------------------
 * Every scene has its own points, cameras, maps (own W x H and view count)
 * and outputs; all use params' search settings and map dtype (params->width,
 * height and depth_maps are ignored: each scene brings its own).  The scenes array is host memory holding device
 * pointers; at most FD_MAX_BATCH_SCENES scenes.  The context is required and
 * must be reserved for the total point count and the scene count.  The
 * launch sequence is captured into a HIP graph on the first call and
 * replayed while the scene array and params are unchanged (a changed array
 * re-captures, which synchronises params->stream).  The learned form takes
 * the network proposal only; FD_MODE_FPMVO is not batched (FD_E_INVAL).  Results equal those of fd_fuse_directions on
 * each scene alone, bit for bit. */
typedef struct fd_scene {
  const float* points;
  int64_t n_points;
  const fd_camera* cams;
  int32_t n_views;
  int32_t width, height;
  const void* orient_maps;
  const void* conf_maps;
  const void* depth_maps;  /* as fd_params.depth_maps, per scene (NULL: no test) */
  float* dirs;
  float* costs;
  float head_centre[3];
  /* learned mode with params->proposal == FD_PROPOSAL_GIVEN: device,
   * n_points x 3 float proposals in point order (a row that is not a finite
   * non-zero direction falls back); otherwise ignored (may be NULL) */
  const float* proposal_dirs;
} fd_scene;

int fd_fuse_directions_batched(const fd_scene* scenes, int32_t n_scenes,
                               const fd_params* params, fd_context* ctx);

/* ---- learned proposal: 112 -> 256 -> 256 -> 256 -> 3 MLP ------------------
 * GELU (tanh form) after the three hidden layers, output normalised.
 * Weights: float master copy (Adam state beside it) and a bfloat16 copy the
 * matrix-core kernels read; activations bfloat16, accumulation float.
 * Flat parameter order (161283 floats): W1[112][256], b1[256], W2[256][256],
 * b2, W3[256][256], b3, W4[256][3], b4[3] with y = x W + b. */
#define FD_MLP_N_PARAMS 161283

typedef struct fd_adam {
  float lr, beta1, beta2, eps;
} fd_adam;

int fd_mlp_create(fd_mlp** out, uint64_t seed);
int fd_mlp_set_params(fd_mlp* mlp, const float* host_params);
int fd_mlp_get_params(const fd_mlp* mlp, float* host_params);
int fd_mlp_set_calibration(fd_mlp* mlp, float learned_step0, float fallback_cost);
int fd_mlp_get_calibration(const fd_mlp* mlp, float* learned_step0, float* fallback_cost);
/* Checkpoint: header, float master weights, Adam moments, step count,
 * calibration.  Little-endian binary file. */
int fd_mlp_save(const fd_mlp* mlp, const char* path);
int fd_mlp_load(fd_mlp* mlp, const char* path);
/* feats: device batch x 112 bfloat16 (raw 16-bit); out: device batch x 3
 * float unit directions. */
int fd_mlp_forward(const fd_mlp* mlp, const void* feats, int64_t batch,
                   float* out, void* stream);
/* Loss and gradient of the mean axial loss 1 - (y . t)^2 over a batch
 * (batch <= 65536): grad device FD_MLP_N_PARAMS floats, loss device float. */
int fd_mlp_loss_grad(fd_mlp* mlp, const void* feats, const float* targets,
                     int32_t batch, float* grad, float* loss, void* stream);
/* One Adam step on the loss of the batch; loss (device float) may be NULL. */
int fd_mlp_train_step(fd_mlp* mlp, const void* feats, const float* targets,
                      int32_t batch, const fd_adam* opt, float* loss,
                      void* stream);
void fd_mlp_destroy(fd_mlp* mlp);

/* Proposal-network input of every point: the FD_FEATURE_SLOTS most frontal
 * eligible views (in front, inside the image and, with params->depth_maps,
 * visible; ranked by the largest cosine between the point->camera direction and
 * p - params->head_centre), each (q_x, q_y, C, v_x, v_y, v_z, valid):
 * v is the unit point->camera direction, C the bilinear confidence and
 * (q_x, q_y) = |m| (cos 2psi, sin 2psi), where m is the bilinear
 * confidence-weighted doubled-angle vector (Eq. 9's orientation sample) and
 * psi the angle, in the frame e1 = normalize(z x v), e2 = v x e1, of the
 * direction across v of the plane that the observed image orientation
 * back-projects to; empty slots are 0.  feats: device n_points x 112
 * bfloat16 (16-byte aligned). */
int fd_features(const float* points, int64_t n_points, const fd_camera* cams,
                int32_t n_views, const void* orient_maps,
                const void* conf_maps, const fd_params* params, void* feats);

/* ---- orientation and confidence maps from frames ---------------------------
 * The paper extracts its maps O and C with Gabor filters (Sec. 3.1, opening
 * paragraph) without giving parameters; the reading: n_orient even (cosine)
 * Gabor kernels of radius r at theta_i = i pi / n_orient (strand direction,
 * from image +x towards +y), exp(-a^2/(2 s_a^2) - b^2/(2 s_b^2))
 * cos(2 pi b / lambda) with a along and b across the direction, made zero
 * mean over the (2r+1)^2 window; response F_i = |correlation| (frame read
 * as 0 outside); theta = theta_{argmax F_i} (first of equals); confidence
 * w = sqrt(sum_i d(theta_i, theta)^2 (F_i - F_max)^2) (d: distance between
 * lines), divided by its maximum over the frame. */
typedef struct fd_gabor_params {
  int32_t n_orient;        /* 8, 16 or 32 */
  int32_t radius;          /* 1..12 */
  float sigma_along;       /* > 0, pixels */
  float sigma_across;      /* > 0, pixels */
  float wavelength;        /* > 0, pixels */
  int32_t out_dtype;       /* FD_F32 or FD_F16 maps */
  void* stream;            /* hipStream_t */
  fd_context* ctx;         /* workspace; NULL = the per-device default */
} fd_gabor_params;

/* Defaults: 32 orientations, radius 8, s_a = 2.4, s_b = 1.8, lambda = 4,
 * FD_F16 output. */
void fd_gabor_params_init(fd_gabor_params* params);

/* frames: device n_frames x H x W float (grey levels, finite), caller-owned;
 * theta_out, conf_out: device n_frames x H x W of params->out_dtype, written
 * (theta radians in [0, pi), conf in [0, 1]).  These are the maps
 * fd_fuse_directions reads.  0 <= n_frames <= FD_MAX_VIEWS,
 * 1 <= W, H <= 32768, at most 2^34 pixels; otherwise FD_E_INVAL and nothing
 * is launched.  The bank (rebuilt when its parameters change, after
 * synchronising the stream), the raw confidences (4 B per pixel) and the
 * frame maxima live in the context's workspace, grown on demand.
 * Asynchronous on params->stream. */
int fd_orientation_maps(const float* frames, int32_t n_frames, int32_t width, int32_t height,
                        const fd_gabor_params* params, void* theta_out, void* conf_out);

/* ---- occupancy and orientation volume --------------------------------------
 * The paper fuses the outer points (with the directions found above) and
 * the inner points into one occupancy / orientation volume before growing
 * strands (Sec. 3.2, opening paragraph) and gives no rule.  The reading:
 *   voxel   point p is in voxel (ix, iy, iz), i_a = floor((p_a - o_a) / h)
 *           with the subtraction and the division in binary32 (IEEE), if
 *           0 <= i_a < dims_a on every axis; linear index
 *           (iz * ny + iy) * nx + ix.  Points outside are ignored.
 *   occupancy  the number of points in the voxel.
 *   orientation  directions are lines, so they are averaged through the
 *           structure tensor T = sum w_i d_i d_i^T of the voxel's points;
 *           the orientation is the unit eigenvector of T's largest
 *           eigenvalue l1 (sign: z > 0, else y > 0, else x >= 0) and the
 *           coherence (l1 - l2) / l1 (1: one direction; 0: spread evenly in
 *           a plane or in space).  A voxel without a weighted direction gets
 *           orientation 0 and coherence 0.
 * Each term w d_a d_b is formed in binary64 from the binary32 inputs, kept
 * in [-1, 1] and rounded to a multiple of 2^-32; the sums are 64-bit
 * integers, so the volume does not depend on the order of the points
 * (deterministic), and each sum is within n_v * 2^-33 of the exact one.
 * The eigenvector is found in binary64 (cyclic Jacobi). */
#define FD_MAX_VOLUME_DIM 4096
#define FD_MAX_VOLUME_VOXELS (1LL << 30)
#define FD_MAX_VOLUME_POINTS ((1LL << 31) - 1)

typedef struct fd_volume_grid {
  float origin[3];   /* world position of the low corner of voxel (0, 0, 0) */
  float voxel;       /* voxel edge h (same unit as the points), finite, > 0 */
  int32_t dims[3];   /* nx, ny, nz in [1, FD_MAX_VOLUME_DIM], product
                        <= FD_MAX_VOLUME_VOXELS */
} fd_volume_grid;

/* points, dirs: device n_points x 3 float (dirs unit or 0; a zero direction
 * counts for the occupancy only); weights: device n_points float in [0, 1]
 * (the point's reliability; values above 1 are taken as 1, below 0 or NaN
 * as 0), or NULL for all 1.  Outputs (device, caller-owned, all written):
 * occ_out nv uint32, dir_out nv x 3 float, coherence_out nv float, and
 * tensor_out nv x 6 double (xx, yy, zz, xy, xz, yz: the fixed-point sums)
 * or NULL.  nv = nx * ny * nz.  The workspace (a counting sort of the
 * points by voxel: 56 B per point, 4 B per voxel) lives in the context,
 * grown on demand.  FD_E_INVAL for a bad grid, size or
 * pointer, with nothing launched.  Asynchronous on stream. */
int fd_fuse_volume(const float* points, const float* dirs, const float* weights,
                   int64_t n_points, const fd_volume_grid* grid, void* stream, fd_context* ctx,
                   uint32_t* occ_out, float* dir_out, float* coherence_out, double* tensor_out);

/* ---- parallel hair growing -------------------------------------------------
 * Strands grow through the volume above from many seeds at once, with the
 * occupancy bookkeeping deferred to the end of each batch (Sec. 3.2.1), and
 * short pieces are joined by the proximity and direction test of Eq. (13)
 * (Sec. 3.2.2).  The paper gives no step, stopping rule, thresholds or
 * conflict rule; the reading:
 *   trace   from seed x_0 with reference r (the seed direction, or the
 *           volume orientation at the seed pointed away from / towards
 *           `centre`).  Step k reads the voxel v of x_{k-1} and stops if
 *           x_{k-1} is outside the grid, v is empty, has coherence below
 *           min_coherence, no orientation, or (voxel_cap > 0) was crossed
 *           voxel_cap times or more by strands of earlier batches.  The
 *           direction t is v's orientation, negated if t.r < 0; from the
 *           second step on the trace also stops if t.r < max_bend_cos (the
 *           first step may leave the seed direction at any angle: a root's
 *           reference is the scalp normal).  x_k = x_{k-1} + step t, r = t.
 *           Binary32 throughout: t.r is a0*b0, then fma(a1, b1, .), then
 *           fma(a2, b2, .); each coordinate is fma(step, t_a, x_a).
 *   batches seeds in order, `batch` at a time; a batch sees the crossing
 *           counts left by the earlier batches (and the caller); after it,
 *           each of its steps adds 1 to the count of the voxel it read.
 *   link    piece i may be continued by piece j != i (flags: bit 0 valid,
 *           bit 1 accepts a predecessor; j needs both) if
 *           |e_i - s_j|^2 < max_dist^2 (binary32: dx*dx, then fma(dy, dy,
 *           .), then fma(dz, dz, .), e_i - s_j per coordinate) and
 *           <u_i, w_j> > min_cos (as t.r above), with e_i, u_i the end point
 *           and direction of i and s_j, w_j the start point and direction of
 *           j, both oriented root to tip.  Each i proposes its nearest such
 *           j (then the lowest j); each j accepts its nearest proposer (then
 *           the lowest i): succ[i] = j for accepted pairs, else -1. */
#define FD_MAX_GROW_STEPS 4096
#define FD_MAX_GROW_SEEDS (1 << 26)
#define FD_MAX_LINK_PIECES (1 << 26)
enum { FD_SEED_GIVEN = 0, FD_SEED_AWAY = 1, FD_SEED_TOWARDS = 2 };

typedef struct fd_grow_params {
  float step;            /* step length (grid unit), finite, > 0 */
  int32_t max_steps;     /* 1..FD_MAX_GROW_STEPS */
  float min_coherence;   /* finite */
  float max_bend_cos;    /* finite; cos of the largest turn between steps */
  int32_t voxel_cap;     /* >= 0; 0 = crossings never stop a trace */
  int32_t batch;         /* >= 1 seeds per batch */
  int32_t seed_mode;     /* FD_SEED_GIVEN (seed_dirs), FD_SEED_AWAY, FD_SEED_TOWARDS */
  float centre[3];       /* for FD_SEED_AWAY / FD_SEED_TOWARDS */
  void* stream;          /* hipStream_t */
  fd_context* ctx;       /* NULL = the per-device default */
} fd_grow_params;

/* Defaults: step 1 mm, 200 steps, min_coherence 0.2, 30 degrees of bend,
 * voxel_cap 8, batch 4096, FD_SEED_GIVEN, centre 0. */
void fd_grow_params_init(fd_grow_params* params);

/* grid, occ, dir, coherence: a volume as fd_fuse_volume writes it (device).
 * seeds: device n_seeds x 3; seed_dirs: device n_seeds x 3 (FD_SEED_GIVEN
 * only, else ignored).  crossings: device nv uint32, read and updated
 * (zero it for a fresh start).  Outputs (device, caller-owned): verts
 * n_seeds x (max_steps + 1) x 3 (entries past n_verts[i] are not written),
 * n_verts n_seeds (>= 1: the seed itself), last_dir n_seeds x 3 (the last
 * step's direction, negated for FD_SEED_TOWARDS so that a backward trace
 * reports the direction root to tip; 0 without a step).  FD_E_INVAL for a
 * bad grid, parameter, size or pointer, with nothing launched.
 * Asynchronous on params->stream (2 launches per batch). */
int fd_grow_strands(const fd_volume_grid* grid, const uint32_t* occ, const float* dir,
                    const float* coherence, const float* seeds, const float* seed_dirs,
                    int32_t n_seeds, const fd_grow_params* params, uint32_t* crossings,
                    float* verts, int32_t* n_verts, float* last_dir);

/* starts, start_dirs, ends, end_dirs: device n x 3 float (finite); flags:
 * device n uint8; succ: device n int32 (written).  max_dist finite, > 0;
 * min_cos finite.  Workspace (2^20 bucket counts and offsets, 28 B per
 * piece) in the context, grown on demand.  FD_E_INVAL for a bad size,
 * threshold or pointer.  Asynchronous on stream. */
int fd_link_segments(const float* starts, const float* start_dirs, const float* ends,
                     const float* end_dirs, const uint8_t* flags, int32_t n, float max_dist,
                     float min_cos, void* stream, fd_context* ctx, int32_t* succ);

/* Strands from linked pieces.  Piece g < n_guide is guide trace g (from
 * fd_grow_strands with the scalp roots); piece n_guide + s is segment s,
 * made of backward trace s (FD_SEED_TOWARDS) reversed without its seed,
 * then forward trace s (FD_SEED_AWAY) from the same seed; succ (n_guide +
 * n_seg, from fd_link_segments over pieces in that order) chains them.
 * Strand g is guide trace g followed by its chain of segments, which ends
 * at -1, at a guide piece, or after n_guide + n_seg links.
 * fd_strand_offsets: offsets (device, n_guide + 1 int64; offsets[n_guide]
 * is the total vertex count) and optionally pieces (device, n_guide int32,
 * pieces per strand).  fd_assemble_strands: out (device, capacity x 3
 * float) receives strand g's vertices at rows offsets[g] ..
 * offsets[g + 1] - 1; rows at or beyond capacity are not written.  Vertex
 * counts must not exceed their stride (max_steps + 1 of the call that
 * traced them), as fd_grow_strands writes them.  FD_E_INVAL for bad sizes
 * or pointers.  Asynchronous on stream. */
int fd_strand_offsets(const int32_t* guide_n, int32_t n_guide, const int32_t* fwd_n,
                      const int32_t* bwd_n, int32_t n_seg, const int32_t* succ, void* stream,
                      fd_context* ctx, int64_t* offsets, int32_t* pieces);
int fd_assemble_strands(const float* guide_v, const int32_t* guide_n, int32_t n_guide,
                        int32_t g_stride, const float* fwd_v, const int32_t* fwd_n,
                        int32_t f_stride, const float* bwd_v, const int32_t* bwd_n,
                        int32_t b_stride, int32_t n_seg, const int32_t* succ,
                        const int64_t* offsets, int64_t capacity, void* stream, fd_context* ctx,
                        float* out);

/* ---- tuning ---------------------------------------------------------------
 * Times the batched launch on the sample scenes for each shape of the
 * plain search (persistent: tiles per queue pop and resident grid size; or
 * one wave per tile) and keeps the fastest in the context (the sample's
 * outputs are overwritten).  With cache_path, a shape class (patch, top_k,
 * map dtype, mode, point-count octave) already in that JSON file is taken
 * from it without timing, and a newly timed one is added to it.  Offline: it
 * synchronises and is not meant for timed regions.  Tile shapes never change
 * results. */
int fd_autotune(fd_context* ctx, const fd_scene* sample, int32_t n_scenes,
                const fd_params* params, const char* cache_path);

/* The tile shape the batched search of this context uses: *chunk tiles per
 * queue pop and *grid workgroups (0: the full resident grid, -1: one wave
 * per tile instead of the persistent queue). */
int fd_tuned_shape(const fd_context* ctx, int32_t* chunk, int32_t* grid);
/* Sets that shape directly (a shape fd_autotune returned for another form,
 * say): chunk >= 1, grid >= 0 (0: the full resident grid) or -1; results
 * do not depend on it.  Returns FD_E_INVAL for other values. */
int fd_set_tuned_shape(fd_context* ctx, int32_t chunk, int32_t grid);

/* ---- stage timing -----------------------------------------------------------
 * While enabled on a context, every call through it records a pair of HIP
 * events on its stream around each stage's kernels.  fd_profile_read waits
 * for the recorded events and returns the summed GPU time (ms) and the
 * number of timed launches of one stage; fd_profile_enable also clears.
 * A batched call made while timing is on launches its kernels directly
 * instead of replaying its graph (a graph holds no event records), so each
 * of its stages is timed; its results are the same. */
enum {
  FD_STAGE_TILING = 0,    /* spatial key, counting sort */
  FD_STAGE_TOPK = 1,      /* Eq. (4) view selection */
  FD_STAGE_FUSE = 2,      /* plain search: patch, lattice, refinement */
  FD_STAGE_FEATURES = 3,  /* proposal-network input */
  FD_STAGE_MLP = 4,       /* proposal network */
  FD_STAGE_REFINE = 5,    /* learned: refinement from the proposal, threshold */
  FD_STAGE_FALLBACK = 6,  /* learned: plain search of the fallback list */
  FD_STAGE_BATCHED = 7,   /* persistent batched launch */
  FD_STAGE_GABOR = 8,     /* orientation maps: filter bank, argmax, raw confidence */
  FD_STAGE_GABOR_NORM = 9, /* orientation maps: confidence normalisation */
  FD_STAGE_VOLUME_CLEAR = 10,   /* volume: zero the counts */
  FD_STAGE_VOLUME_SCATTER = 11, /* volume: voxel keys, counts, scan, sort by voxel */
  FD_STAGE_VOLUME_FINAL = 12,   /* volume: per-voxel sums, eigenvector, coherence */
  FD_STAGE_GROW = 13,           /* growing: one batch of traces */
  FD_STAGE_GROW_CROSS = 14,     /* growing: the batch's deferred crossing counts */
  FD_STAGE_LINK = 15,           /* segment linking (all its kernels) */
  FD_N_STAGES = 16
};
int fd_profile_enable(fd_context* ctx, int on);
int fd_profile_read(fd_context* ctx, int stage, double* total_ms, int64_t* count);

/* ---- bandwidth probe (measurement) -------------------------------------------
 * Reads the device buffer buf (bytes, a multiple of 16, at most 2^31) reps
 * times from every one of `blocks` workgroups of 256 lanes (each workgroup
 * walks the whole buffer with 16-byte loads), folds what it read into one
 * 32-bit value per lane and writes those to sink (device, blocks x 256
 * uint32, caller-owned).  A buffer that fits one XCD's L2 (4 MiB) is then
 * read from L2 by every XCD, so bytes x reps x blocks over the kernel time
 * is the aggregate L2 read bandwidth; a much larger buffer measures HBM.
 * Enqueued on stream (NULL: the null stream); no allocation.  Returns
 * FD_E_INVAL for a null pointer, bytes not a positive multiple of 16 or
 * above 2^31, reps < 1 or blocks < 1. */
int fd_probe_read(const void* buf, int64_t bytes, int32_t reps, int32_t blocks, uint32_t* sink,
                  void* stream);

const char* fd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
