/*
 * romap.h -- C ABI of the MI355X (gfx950) training path for RO-MAP's
 * per-object radiance fields (Han, Yang et al., "RO-MAP: Real-Time
 * Multi-Object Mapping with Neural Radiance Fields", arXiv 2304.05735).
 *
 * The verbs follow the paper's statement of the problem:
 *  - a new object instance gets its own model: a multiresolution hash
 *    encoding plus a small MLP (Sec. V), registered with its cuboid box
 *    (centre t, yaw theta, half size a: Sec. IV-B, Eq. 1 and Eq. 4);
 *  - posed keyframes with instance masks (and sparse depth) arrive over time
 *    and join an object's training set by the view-angle rule of Eq. 5
 *    (Sec. V-A "Data");
 *  - objects train for a number of iterations on new observations and stop
 *    when idle (Sec. V-A "Parallel Training", Sec. VI implementation details);
 *  - each iteration draws rays inside the object's detection box, samples
 *    uniformly inside its 3D box, volume-renders (Eq. 6), applies the loss of
 *    Eq. 7-11, backpropagates and updates the parameters (Sec. V-B, Table 3);
 *  - density is queried for meshing, and views are rendered for evaluation.
 *
 * Conventions
 *  - Every call returns romap_status: 0 = ROMAP_OK, negative = error.
 *    Nothing aborts or throws across the ABI.  romap_last_error() gives a
 *    message for the last failing call on a context.
 *  - Arguments are validated before any side effect: a failing call leaves
 *    the context unchanged (except where stated for ROMAP_E_HIP).
 *  - Host buffers are owned by the caller and copied before the call returns.
 *    Pointers documented as device pointers must be device memory of the
 *    current HIP device; work on them is ordered on the context's stream and
 *    is complete once that stream has synchronised.
 *  - One thread at a time per context; several contexts may coexist.
 *  - Cameras are pinhole, x right, y down, z forward, pixel centres at +0.5;
 *    T_wc is the row-major 3x4 camera-to-world pose.  World +z is up; an
 *    object's yaw turns about +z (roll = pitch = 0, Sec. IV-B).
 *  - Parameter order of an object (get/set_params): the grid level-major,
 *    [level][entry][feature] with F = 2 features and level l holding
 *    T_l = min(T, (N_l + 1)^3) entries; then the MLP weights W1 (64 x 2L),
 *    mlp_layers - 1 matrices 64 x 64 of a deeper density MLP, W2 (16 x 64),
 *    W3 (64 x 15), W4 (3 x 64), row-major (row = output), no biases.
 */
#ifndef ROMAP_H
#define ROMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t romap_status;
#define ROMAP_OK 0
#define ROMAP_E_INVALID_ARG (-1)
#define ROMAP_E_OUT_OF_MEMORY (-2)
#define ROMAP_E_NOT_FOUND (-3)
#define ROMAP_E_HIP (-4)
#define ROMAP_E_NUMERIC (-5) /* NaN/Inf in an object's loss */
#define ROMAP_E_STATE (-6)   /* e.g. the object has no keyframe yet */

typedef struct romap_ctx romap_ctx;

#define ROMAP_PREC_FP32 0 /* MLP contractions on FP32 MFMA */
#define ROMAP_PREC_BF16 1 /* MLP contractions on BF16 MFMA, FP32 accumulate */

#define ROMAP_BATCH_ALL 0        /* every object of a step in one launch per phase (two
                                    object groups on two streams with streams = 2) */
#define ROMAP_BATCH_PER_OBJECT 1 /* one launch per object per phase */

/* Model and training hyperparameters.  Defaults: romap_default_config(). */
typedef struct {
  int32_t n_levels;        /* L, 1..16 */
  int32_t base_res;        /* N_min */
  int32_t max_res;         /* N_max */
  int32_t log2_table_size; /* default log2 T for objects registered with 0 */
  int32_t samples_per_ray; /* N: 32, 64 or 128 (uniform samples, Sec. V-B) */
  int32_t rays_per_step;   /* default rays per object per step (4096 in Sec. VI);
                              1..2^22 and rays x samples_per_ray <= 2^27 */
  float lr, beta1, beta2, eps;             /* Adam */
  float lambda_depth, lambda_density;      /* lambda_1, lambda_2 of Eq. 11 */
  float alpha_deg;                         /* keyframe rule threshold of Eq. 5 */
  int32_t bbox_margin_pct;                 /* detection-box margin, % per side */
  int32_t precision;                       /* ROMAP_PREC_* */
  int32_t batch_mode;                      /* ROMAP_BATCH_* */
  int32_t use_graph;                       /* 1: replay each step as one hipGraph
                                            * (captured when the call has >= 8 steps
                                            * or the graph of its shapes exists);
                                            * 2: capture on any training call, so a
                                            * short untimed call prepares the graph;
                                            * 0: launch every kernel */
  int32_t autotune;                        /* pick tile shapes by timing */
  int32_t profile_phases;                  /* time each kernel of a step with HIP
                                              events (launches without a graph and
                                              waits after every step) */
  int32_t mlp_layers;                      /* hidden layers (64 wide) of the density
                                              MLP: 1 (Sec. V), 2 or 3 (the model-size
                                              study of Table 4).  The extra 64 x 64
                                              matrices follow W1 in the parameters */
  int32_t streams;                         /* 2 (default): a batched training step of
                                              two or more objects runs as two groups of
                                              objects (about 3/4 and 1/4 of the work)
                                              on two streams (the context stream and
                                              one of the library's, joined back after
                                              every step), so that their phases
                                              overlap; 1: one stream */
  uint64_t seed;
} romap_config;

typedef struct {
  float t[3];    /* centre in the world (Eq. 1) */
  float yaw;     /* radians about world +z */
  float half[3]; /* half extents a (Eq. 4), > 0 */
} romap_box;

typedef struct {
  float T_wc[12]; /* row-major 3x4 camera-to-world */
  float fx, fy, cx, cy;
  int32_t width, height;
} romap_camera;

typedef struct {
  float loss_mean;        /* mean over objects and steps of the per-object loss */
  int64_t rays_trained;   /* rays drawn in the call, all objects */
  float seconds;          /* GPU time of the call */
  int32_t n_objects_nan;  /* objects whose loss was not finite */
} romap_train_stats;

typedef struct {
  int32_t instance_id;
  int32_t log2_table_size;
  int64_t n_grid_params;
  int64_t n_mlp_params;
  int32_t n_keyframes;
  int32_t step;          /* Adam steps taken */
  int64_t n_candidates;  /* candidate pixels over all its keyframes */
  int32_t active;
  int32_t level_res[16];
  int32_t level_hashed[16];
} romap_object_info;

#define ROMAP_PARAMS 0 /* grid then MLP */
#define ROMAP_ADAM_M 1
#define ROMAP_ADAM_V 2
#define ROMAP_GRAD 3   /* gradient buffer: dL/dparams after romap_loss_and_grad; zero
                        * after romap_train, whose Adam update is applied where each
                        * gradient is complete (the buffer is not written) */

/* Fills *cfg with the defaults: L 16, N_min 16, N_max 1024, T 2^19, N 64,
 * 4096 rays, Adam lr 1e-2 b1 0.9 b2 0.99 eps 1e-15, lambda_1 0.5,
 * lambda_2 0.01 (Sec. VI), alpha 25 deg (Sec. VI), margin 10 %, FP32,
 * batched, graph on, autotune on, seed 0.  Always succeeds for non-NULL cfg. */
romap_status romap_default_config(romap_config* cfg);

/* Creates a context on the current HIP device.  hip_stream: a hipStream_t to
 * order all work on, or NULL for a stream owned by the context.  On success
 * *out owns every device allocation the context makes. */
romap_status romap_create(const romap_config* cfg, void* hip_stream, romap_ctx** out);
romap_status romap_destroy(romap_ctx* ctx);
/* Message of the last failing call on ctx (or of the last failing create if
 * ctx is NULL).  Owned by the library, valid until the next call. */
const char* romap_last_error(const romap_ctx* ctx);

/* Registers an object (Sec. V: a new model when a new instance is detected)
 * with its box and hash table size log2 T in [8, 24] (0 = config default).
 * Parameters start as grid U(-1e-4, 1e-4), MLP Glorot-uniform, drawn from
 * Philox keyed on (seed, object id).  *object_id receives the new id
 * (0, 1, ... in registration order).  Keyframes added earlier are not used. */
romap_status romap_add_object(romap_ctx* ctx, int32_t instance_id, const romap_box* box,
                              int32_t log2_table_size, int32_t* object_id);
/* Idle objects stop training (Sec. V-A): inactive objects are skipped when
 * romap_train is given object_ids = NULL. */
romap_status romap_set_object_active(romap_ctx* ctx, int32_t object_id, int32_t active);
romap_status romap_get_object_info(romap_ctx* ctx, int32_t object_id, romap_object_info* info);

/* Occupancy skip for long ray budgets (not in the paper; used by the
 * incremental mapping stream): a 64^3 bitfield over the object's box, bit
 * x + 64 y + 4096 z (least significant bit first in each byte) for the cell
 * floor(64 p) of a sample at normalised position p (clamped to 0..63).  A
 * sample in a clear cell has density 0: it skips the encoding, adds nothing
 * to rendering, the density loss or the gradient.  Applies to training,
 * rendering and the differentiable surface; not to romap_query_density.
 *   set:    bits = 32768 host bytes, or NULL to switch skipping off
 *   update: bits = (density at the cell centre > threshold), switches it on
 *   get:    copies the bits out (ROMAP_E_STATE if skipping is off) */
romap_status romap_set_occupancy(romap_ctx* ctx, int32_t object_id, const uint8_t* bits);
romap_status romap_update_occupancy(romap_ctx* ctx, int32_t object_id, float threshold);
romap_status romap_get_occupancy(romap_ctx* ctx, int32_t object_id, uint8_t* bits);

/* Adds a posed keyframe (Sec. V-A "Data").  rgb: H*W*3 bytes; mask: H*W
 * int32 instance ids, 0 = background; depth_z: H*W camera z of sparse depth,
 * <= 0 or non-finite = none, may be NULL.  For every registered object seen
 * in the mask the keyframe joins its set if it is the object's first, or if
 * the angle of Eq. 5 to the object's last accepted keyframe exceeds
 * alpha_deg.  *keyframe_id and *n_objects_accepted may be NULL. */
romap_status romap_add_keyframe(romap_ctx* ctx, const romap_camera* cam, const uint8_t* rgb,
                                const int32_t* mask, const float* depth_z, int32_t* keyframe_id,
                                int32_t* n_objects_accepted);

/* Runs n_steps training iterations (draw, render, loss, backward, Adam) on
 * every listed object (NULL = every active object).  rays_per_object: rays
 * per step for each listed object, each in [1, 2^22] with rays x
 * samples_per_ray <= 2^27, at most 2^30 over the list (NULL = config
 * default); any other count is ROMAP_E_INVALID_ARG.  An empty list
 * (n_objects = 0) or n_steps = 0 does nothing and succeeds.  stats may be
 * NULL, in which case the call does not wait for the GPU.  Returns
 * ROMAP_E_STATE if a listed object has no keyframe, ROMAP_E_NUMERIC (after
 * the steps ran) if an object's loss is not finite. */
romap_status romap_train(romap_ctx* ctx, const int32_t* object_ids, int32_t n_objects,
                         int32_t n_steps, const int32_t* rays_per_object,
                         romap_train_stats* stats);

/* One step's loss and gradient without the Adam update or step advance: the
 * gradient buffer is cleared, then holds dL/dparams (read it with kind
 * ROMAP_GRAD).  Objects and ray counts as for romap_train, in one launch per
 * kernel on the context stream with the launch shape a training step of
 * these objects takes (autotuned, or the romap_debug_tiles shape).  losses
 * (host, n_objects floats) may be NULL. */
romap_status romap_loss_and_grad(romap_ctx* ctx, const int32_t* object_ids, int32_t n_objects,
                                 const int32_t* rays_per_object, float* losses);

/* Renders one object's model from a camera (composited on black):
 * rgb H*W*3, depth H*W (ray distance), opacity H*W (1 - T_end); any output
 * may be NULL.  out_on_device: outputs are device pointers (ordered on the
 * context stream) rather than host buffers (the call then waits). */
romap_status romap_render(romap_ctx* ctx, int32_t object_id, const romap_camera* cam, float* rgb,
                          float* depth, float* opacity, int32_t out_on_device);

/* Density at n object-frame points xyz (n*3), for meshing (Sec. III:
 * marching cubes on the object's density).  Points outside the box are
 * clamped to it.  on_device: xyz and sigma are device pointers. */
romap_status romap_query_density(romap_ctx* ctx, int32_t object_id, const float* xyz, int64_t n,
                                 float* sigma, int32_t on_device);

/* An object's box from its sparse world point cloud (Sec. IV-B, pose and
 * size estimation; host computation in FP64, no device needed): t = the
 * midpoint of the per-axis extremes of the points (Eq. 1); yaw = the
 * direction of the dominant principal axis of the points projected on the
 * horizontal plane (PCA of their 2x2 second moments about the mean), folded
 * into [-pi/2, pi/2); half = half the per-axis extent of the points in the
 * object frame, R(yaw)^T (x - t) (Eq. 4).  Roll and pitch are zero.  The
 * paper's refinement of the yaw by image line features (Eq. 2-3) is not
 * computed.  xyz: n*3 floats (host); ROMAP_E_INVALID_ARG if n < 1 or a
 * pointer is NULL.  The result feeds romap_add_object. */
romap_status romap_box_from_points(const float* xyz, int64_t n, romap_box* box);

/* Marching cubes (Sec. III: the object meshes; 64^3 per object in Sec. VI)
 * on a density grid of (res+1)^3 corner values, x fastest, corner (i, j, k)
 * at lo + (hi - lo) * (i, j, k) / res (FP32, that order).  A corner is
 * inside when its value is > iso; the vertex on an edge from corner a to b
 * is x_a + t (x_b - x_a), t = (iso - v_a) / (v_b - v_a).  Triangles come in
 * cell order (x fastest), each cell's as its case lists them (romap_mc_case),
 * oriented with normals pointing from inside to outside.  tris: up to
 * max_tris triangles of 9 floats (three vertices) are written; *n_tris
 * receives the total count (so tris = NULL, max_tris = 0 counts).  grid and
 * tris are device pointers when on_device (the call still waits for the
 * count).  res in 1..160, else ROMAP_E_INVALID_ARG. */
romap_status romap_marching_cubes(romap_ctx* ctx, const float* grid, int32_t res, float iso,
                                  const float lo[3], const float hi[3], float* tris,
                                  int64_t max_tris, int64_t* n_tris, int32_t on_device);

/* An object's mesh: its density (as romap_query_density) on the (res+1)^3
 * corners of its box [-a, a], then romap_marching_cubes at iso; in the
 * object frame, or with world_frame = 1 placed by the box pose,
 * x_w = Rz(yaw) x + t (Sec. III: meshes transformed to the global frame by
 * the object poses).  Buffers and errors as romap_marching_cubes. */
romap_status romap_extract_mesh(romap_ctx* ctx, int32_t object_id, int32_t res, float iso,
                                int32_t world_frame, float* tris, int64_t max_tris,
                                int64_t* n_tris, int32_t on_device);

/* The marching-cubes case table (host only, no device needed): the edge
 * triples of case m (bit c set = corner c inside; corner c at (c&1, c>>1&1,
 * c>>2&1); edges 0-3 along x from corners 0,2,4,6, 4-7 along y from 0,1,4,5,
 * 8-11 along z from 0,1,2,3) into tris[16] (-1 after the last), returns the
 * triangle count.  Built from the cube's faces: on a face with four crossing
 * edges each inside corner is cut off by its two edges; loops oriented by
 * their Newell normal from inside to outside, started at their smallest
 * edge, fanned from the first vertex whose fan has no triangle in a face. */
int32_t romap_mc_case(int32_t m, int8_t tris[16]);

/* Copies an object's parameters (kind ROMAP_PARAMS / ADAM_M / ADAM_V / GRAD)
 * to or from a host buffer of n floats.  *n_required (may be NULL) receives
 * the count; buf may be NULL to query it.  ROMAP_E_INVALID_ARG if n is
 * smaller than the count. */
romap_status romap_get_params(romap_ctx* ctx, int32_t object_id, int32_t kind, float* buf,
                              int64_t n, int64_t* n_required);
romap_status romap_set_params(romap_ctx* ctx, int32_t object_id, int32_t kind, const float* buf,
                              int64_t n);

/* Checkpoint of the whole context: config, objects (box, parameters, Adam
 * state, step counters, keyframe sets) and keyframes.  A loaded context
 * continues bit-identically because every random draw is a Philox counter
 * keyed on (seed, object, step, ray).  load needs an empty context. */
romap_status romap_save(romap_ctx* ctx, const char* path);
romap_status romap_load(romap_ctx* ctx, const char* path);

/* ---- inspection: the drawn rays of one step ------------------------------
 * Draws object_id's rays for its current step exactly as romap_train does
 * and copies them to host arrays (each may be NULL):
 *   kf_uv     n_rays*3 int32: keyframe index within the object's set, u, v
 *   cls       n_rays int32: 0 occluder, 1 object, 2 background (Sec. V-B);
 *             -1 when the ray misses the box
 *   ray_f     n_rays*16 floats: o[3], d[3], t_n, delta, target[3] (image colour,
 *             or the random colour of a background ray), D, 0, 0, 0, has_depth
 *   positions n_rays*N*3 floats: normalised sample positions in [0,1]^3    */
romap_status romap_debug_rays(romap_ctx* ctx, int32_t object_id, int32_t n_rays, int32_t* kf_uv,
                              int32_t* cls, float* ray_f, float* positions);
/* Hash-grid encoding of n normalised positions p (n*3, [0,1]^3) with the
 * object's current grid: idx n*L*8 uint32 corner indices within each level,
 * feat n*L*2 floats.  Host buffers; either output may be NULL. */
romap_status romap_debug_encode(romap_ctx* ctx, int32_t object_id, const float* p, int64_t n,
                                uint32_t* idx, float* feat);
/* For tests of the overflow path of the gradient binning: caps every bin
 * (the records of one 2048-entry table region) at `slots` record slots,
 * rounded up to a multiple of 4 (0 restores the sized capacity).  Records
 * beyond a bin's capacity go to the gradient with atomics and are merged by
 * the region's accumulation: results are the same up to rounding order, the
 * step only slower.  ROMAP_E_INVALID_ARG if slots < 0. */
romap_status romap_debug_bin_capacity(romap_ctx* ctx, int32_t slots);
/* For tests of the launch shapes the autotuner chooses among: with
 * autotune = 0, training steps and romap_loss_and_grad launch the field
 * kernel with `rays_per_item` rays per workgroup (4, 8, 16 or 32) and the
 * gather kernel with `gather_block` samples per block (128, 256 or 512);
 * the defaults are 8 and 256.  Results are the same up to rounding order.
 * ROMAP_E_INVALID_ARG for other values. */
romap_status romap_debug_tiles(romap_ctx* ctx, int32_t rays_per_item, int32_t gather_block);
/* Sustained matrix-core rate of the current device in TFLOP/s, measured by a
 * kernel of independent MFMA chains with no memory traffic, eight waves per
 * SIMD (precision ROMAP_PREC_BF16: 32x32x16 BF16 MFMA; ROMAP_PREC_FP32:
 * 16x16x4 FP32 MFMA): the measured peak beside the datasheet one against which the
 * MLP kernel's rate is stated.  Runs on the null stream and waits for it;
 * allocates and frees a small output buffer.  ROMAP_E_INVALID_ARG for another
 * precision or tflops == NULL, ROMAP_E_HIP / ROMAP_E_OUT_OF_MEMORY on runtime errors. */
romap_status romap_debug_mfma_rate(int32_t precision, double* tflops);

/* ---- differentiable surface (for torch.autograd.Function) ----------------
 * rays_dev: n_rays*8 floats per ray: origin[3], unit direction[3], t_near,
 * t_far, in the object frame (t_far <= t_near = empty ray).  params_dev: the
 * object's parameter vector in ROMAP_PARAMS order (NULL = the object's own).
 * Forward writes rgb (n*3, on black), depth (n) and T_end (n); any may be
 * NULL.  Backward recomputes every per-sample activation (nothing is stored
 * between the calls) and writes dL/dparams into d_params_dev (overwritten),
 * given dL/drgb, dL/ddepth, dL/dT_end (any may be NULL = zero).  All
 * pointers are device pointers ordered on the context stream.  n_rays as
 * for romap_train (1..2^22, n_rays x samples_per_ray <= 2^27), else
 * ROMAP_E_INVALID_ARG. */
romap_status romap_field_forward(romap_ctx* ctx, int32_t object_id, const float* params_dev,
                                 const float* rays_dev, int32_t n_rays, float* rgb_dev,
                                 float* depth_dev, float* tend_dev);
romap_status romap_field_backward(romap_ctx* ctx, int32_t object_id, const float* params_dev,
                                  const float* rays_dev, int32_t n_rays, const float* d_rgb_dev,
                                  const float* d_depth_dev, const float* d_tend_dev,
                                  float* d_params_dev);

/* For callers that cannot allocate device memory (code being captured into
 * a graph, tight serving loops, harnesses that forbid allocation): the same
 * result as romap_field_forward (same kernels and launch shape, bit for bit)
 * with no allocation of any kind on the device.  Its rays, encodings, packed
 * weights and work tables live in one 64 MiB array of the library on each
 * GPU, held until the process ends; a call needs 64 B per ray, 8 L B per
 * sample (L levels, samples_per_ray samples per ray) and small tables, at
 * most 64 MiB: about 8100 rays at 16 levels and 64 samples, 4000 at 128.
 * Larger calls return ROMAP_E_INVALID_ARG with the size in the message.
 * Calls on one GPU share that array: calls that overlap in time on one GPU
 * (several contexts, several host threads, several streams) race and give
 * wrong results.  Returns after the kernels are queued and the work tables
 * copied (it waits for the context stream).  Arguments as for
 * romap_field_forward. */
romap_status romap_field_forward_noalloc(romap_ctx* ctx, int32_t object_id,
                                         const float* params_dev, const float* rays_dev,
                                         int32_t n_rays, float* rgb_dev, float* depth_dev,
                                         float* tend_dev);

/* Kernels of one training step, in launch order. */
#define ROMAP_PHASE_RAYGEN 0      /* ray draw, classification, box clipping (Sec. V-B) */
#define ROMAP_PHASE_ENCODE 1      /* hash-grid gather */
#define ROMAP_PHASE_PACK 2        /* MLP weights -> MFMA operand images, step advance */
#define ROMAP_PHASE_FIELD 3       /* MLP, volume rendering, loss, adjoint */
#define ROMAP_PHASE_REDUCE 4      /* per-object MLP gradient and loss; Adam on the MLP */
#define ROMAP_PHASE_BIN_SCATTER 5 /* hash-grid gradient: records sorted into bins */
#define ROMAP_PHASE_BIN_ACC 6     /* hash-grid gradient: bin sums; Adam on the table */
#define ROMAP_PHASE_BIN_FINISH 7  /* Adam on table regions summed by several groups */
#define ROMAP_N_PHASES 8

/* Average duration in ms of each kernel of a step (summed over its launches
 * within the step) over the steps of the last romap_train call made with
 * profile_phases = 1 (measured with HIP events on the context stream).  avg_ms: ROMAP_N_PHASES floats.  *n_steps (may be
 * NULL) receives the number of steps averaged (0 if none). */
romap_status romap_get_phase_times(romap_ctx* ctx, float* avg_ms, int32_t* n_steps);
/* Gradient records per step (written by the binning kernel, read by the
 * accumulation; 8 B each) averaged over the same profiled steps: the work
 * measure of the two binning kernels (fewer than 8 per sample and level
 * where runs of samples in one cell are merged). */
romap_status romap_get_step_records(romap_ctx* ctx, double* avg_records);

/* Synchronises the context stream. */
romap_status romap_sync(romap_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
