/*
 * romap_oracle.h -- declarations of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the GPU
 * library is checked against.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Values are FP64.  The ray / sample-position / hash-index path is IEEE FP32
 * with a fixed expression order (no FMA contraction), so that positions and
 * indices can be compared bit for bit.
 */
#ifndef ROMAP_ORACLE_H
#define ROMAP_ORACLE_H
#include <stdint.h>

#define OR_MAX_LEVELS 16
#define OR_HIDDEN 64
#define OR_GEO 15
#define OR_DOUT 16 /* 1 density logit + 15 geometry features */
#define OR_MAX_MLP_LAYERS 3 /* hidden layers of the density MLP (Table 4: 1, 2, 3) */

typedef struct {
  int32_t L, nmin, nmax, log2T, N; /* levels, coarsest/finest res, log2 table, samples per ray */
  int32_t margin_pct;              /* detection-box margin, percent of box size per side */
  double lambda_depth, lambda_density;
  double lr, beta1, beta2, eps;
  uint64_t seed;
} or_config;

typedef struct {
  int32_t L;
  int32_t N[OR_MAX_LEVELS];      /* integer grid resolution of each level */
  int64_t T[OR_MAX_LEVELS];      /* entries of each level */
  int32_t hashed[OR_MAX_LEVELS]; /* 1 = spatial hash, 0 = dense 1:1 */
  int64_t off[OR_MAX_LEVELS + 1];/* offset of each level in floats (F = 2) */
  int32_t mlp_layers;            /* hidden layers of the density MLP, 1..3 (1 from
                                    or_make_levels; the caller may raise it) */
  int32_t mlp_bf16;              /* 1: BF16 mode of the MLP contractions (see or_bf16);
                                    0 from or_make_levels */
} or_levels;

typedef struct {
  const uint8_t* rgb;  /* H*W*3 */
  const int32_t* mask; /* H*W, 0 = background */
  const float* depth;  /* H*W camera z, <= 0 or non-finite = none; may be NULL */
  int32_t W, H;
  float fx, fy, cx, cy;
  float M[9], c[3];         /* camera -> object frame (rotation, camera centre) */
  int32_t x0, y0, w, h;     /* candidate rectangle for this object */
} or_keyframe;

typedef struct {
  int32_t kf, u, v, cls, hit, has_depth; /* cls: 0 occluder, 1 object, 2 background */
  float C[3], Crand[3], D;
  float o[3], d[3], tn, tf, delta;
  double Chat[3], Dhat, Tend, loss;
} or_ray;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int or_make_levels(int L, int nmin, int nmax, int log2T, or_levels* out);
int64_t or_grid_params(const or_levels* lv);
int64_t or_mlp_params(int din, int layers);
void or_object_frame(const float Twc[12], const float t[3], float yaw, float M[9], float c[3]);
void or_pixel_ray(const float M[9], const float c[3], float fx, float fy, float cx, float cy,
                  int u, int v, float o[3], float d[3]);
int or_slab(const float o[3], const float d[3], const float half[3], float* tn, float* tf);
void or_sample_positions(const float o[3], const float d[3], const float half[3], float tn,
                         float tf, int N, float* delta, float* dist, float* pos);
void or_encode(const or_levels* lv, const float p[3], const double* grid, uint32_t* idx,
               double* w, double* e);
double or_bf16(double x);
double or_bf16_gap(double x);
void or_bf16_set_jitter(double rel); /* tests only */
void or_set_tie_jitter(double rel);  /* tests only */
void or_set_jitter_seed(uint64_t seed); /* tests only */
void or_mlp_forward(int din, int layers, int bf16, const double* mlp, const double* e, double* h1,
                    double* y, double* h2, double* sigma, double* rgb, double* rgbc);
void or_composite(int N, const double* sigma, const double* rgb, const double* dist, double delta,
                  int background, const double crand[3], double C[3], double* D, double* Tend,
                  double* w);
int or_candidate_rect(const int32_t* mask, int W, int H, int instance, int margin_pct,
                      int32_t rect[4]);
void or_draw_ray(const or_config* cfg, int obj, int step, int r, int nkf, const or_keyframe* kfs,
                 int instance, or_ray* out);
int or_object_step(const or_config* cfg, const or_levels* lv, int obj, int instance,
                   const float half[3], int nkf, const or_keyframe* kfs, int step, int B,
                   const double* params, const uint8_t* occ, double* grad, double* grad_abs,
                   double* ambiguous, double* bf16_allow, double* min_margin, double* loss,
                   double* loss_allow, or_ray* rays, int nthreads);
int or_field(const or_config* cfg, const or_levels* lv, const float half[3], const double* params,
             int n, const float* rays, double* rgb, double* depth, double* tend,
             const double* d_rgb, const double* d_depth, const double* d_tend, double* grad,
             double* grad_abs, double* ambiguous, double* bf16_allow, int nthreads);
void or_adam(int64_t P, double* p, double* g, double* m, double* v, int k, double lr, double b1,
             double b2, double eps);
int or_render(const or_config* cfg, const or_levels* lv, const float half[3],
              const or_keyframe* cam, const double* params, const uint8_t* occ, double* rgb,
              double* depth, double* opacity, double* rgb_allow, int nthreads);
int or_occupied(const uint8_t* occ, const float p[3]);
void or_query_density(const or_levels* lv, const float half[3], const double* params, int64_t n,
                      const float* xyz, double* sigma);
int or_mc_case(int m, int8_t tris[16]);
int64_t or_marching_cubes(const float* grid, int res, float iso, const float lo[3],
                          const float hi[3], float* out, int64_t max_tris);
int or_box_from_points(const double* xyz, int64_t n, double t[3], double* yaw, double half[3]);

#endif
