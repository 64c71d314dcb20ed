/*
 * romap_oracle.c -- plain CPU oracle for one training step of RO-MAP's
 * per-object radiance fields (arXiv 2304.05735, Sec. V "Multi-Object
 * Reconstruction System").
 *
 * TEST INFRASTRUCTURE ONLY.  The GPU library is checked against this file.
 * It shares no code with the GPU library, and nothing on the product path
 * may load it.  It is written for clarity, not speed: one ray at a time, one
 * sample at a time, in the order the paper states the steps.
 *
 * Precision: every value is FP64, except the ray / slab / sample-position /
 * hash-index path, which is IEEE FP32 in the fixed expression order written
 * below (build with -ffp-contract=off).  That path decides integers (grid
 * cells, hash indices), so both sides must take those decisions in the same
 * precision.  A BF16 mode of the MLP (or_levels.mlp_bf16) rounds every
 * operand of an MLP contraction to BF16 and keeps the rest FP64 (or_bf16).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *  - hash grid: the multiresolution hash encoding the paper cites
 *    (Mueller et al. 2022): per level resolution N_l, dense 1:1 indexing when
 *    (N_l+1)^3 <= T, otherwise XOR of coordinate * {1, 2654435761, 805459861}
 *    modulo T; trilinear blend of F = 2 features;
 *  - N_l = floor(N_min * b^l + 1e-6), b = exp((ln N_max - ln N_min)/(L-1));
 *  - the box maps to the unit cube anisotropically, p = (x + a) / (2a),
 *    clamped to [0,1];
 *  - uniform sampling (Sec. V-B) places N midpoints in [t_n, t_f] with equal
 *    spacing delta, and every sample uses delta (the last one too);
 *  - sigma = exp(min(y0, 15)); no MLP biases; colour = sigmoid;
 *  - background rays composite the residual transmittance against their
 *    random colour, object rays composite on black (Eq. 6, Eq. 9);
 *  - L_rgb and L_rr use the squared per-channel error; every ray term is
 *    divided by the number of rays drawn for the object;
 *  - optimiser: dense Adam (the paper does not name its optimiser).
 */
#include "romap_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 * The paper draws its 4096 rays "randomly" from all training images and gives
 * background rays random colours (Sec. V-B, Sec. VI implementation details);
 * Philox makes every draw a pure function of (seed, object, step, ray). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u; /* golden ratio */
      k1 += 0xBB67AE85u; /* sqrt(3) - 1 */
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Level table of the multiresolution hash encoding (Sec. V: each object model
 * is a hash encoding plus a small MLP; table size T and finest resolution are
 * the model parameters of Sec. VI). */
int or_make_levels(int L, int nmin, int nmax, int log2T, or_levels* out) {
  if (L < 1 || L > OR_MAX_LEVELS || nmin < 1 || nmax < nmin || log2T < 4 || log2T > 24)
    return -1;
  memset(out, 0, sizeof(*out));
  out->L = L;
  double b = 1.0;
  if (L > 1) b = exp((log((double)nmax) - log((double)nmin)) / (double)(L - 1));
  int64_t T = (int64_t)1 << log2T;
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    int N = (L > 1) ? (int)floor((double)nmin * pow(b, (double)l) + 1e-6) : nmin;
    int64_t dense = (int64_t)(N + 1) * (N + 1) * (N + 1);
    out->N[l] = N;
    out->hashed[l] = dense > T;
    out->T[l] = dense > T ? T : dense;
    out->off[l] = off;
    off += out->T[l] * 2;
  }
  out->off[L] = off;
  out->mlp_layers = 1;
  return 0;
}

int64_t or_grid_params(const or_levels* lv) { return lv->off[lv->L]; }

/* W1 (64 x din), then layers - 1 hidden-to-hidden matrices Wh (64 x 64) of
 * the density MLP, W2 (16 x 64), W3 (64 x 15), W4 (3 x 64); row-major (row =
 * output), no biases */
int64_t or_mlp_params(int din, int layers) {
  return (int64_t)OR_HIDDEN * din + (int64_t)(layers - 1) * OR_HIDDEN * OR_HIDDEN +
         OR_DOUT * OR_HIDDEN + OR_HIDDEN * OR_GEO + 3 * OR_HIDDEN;
}

/* ------------------------------------------------------------------------ */
/* Camera pose into the object frame (Sec. V-B: "transform the camera pose to
 * the object coordinate system").  Objects have roll = pitch = 0 and a yaw
 * theta about the world up axis, centre t (Sec. IV-B, Eq. 1); the camera pose
 * T_wc maps camera to world (Eq. 3).  x_obj = R(theta)^T (R_wc x_cam + t_wc - t),
 * so M = R^T R_wc and c = R^T (t_wc - t), computed in FP64, rounded once. */
void or_object_frame(const float Twc[12], const float t[3], float yaw, float M[9], float c[3]) {
  double ct = cos((double)yaw), st = sin((double)yaw);
  for (int j = 0; j < 3; ++j) {
    double r0 = (double)Twc[0 * 4 + j], r1 = (double)Twc[1 * 4 + j], r2 = (double)Twc[2 * 4 + j];
    M[0 * 3 + j] = (float)(ct * r0 + st * r1);
    M[1 * 3 + j] = (float)(-st * r0 + ct * r1);
    M[2 * 3 + j] = (float)r2;
  }
  double dx = (double)Twc[3] - (double)t[0];
  double dy = (double)Twc[7] - (double)t[1];
  double dz = (double)Twc[11] - (double)t[2];
  c[0] = (float)(ct * dx + st * dy);
  c[1] = (float)(-st * dx + ct * dy);
  c[2] = (float)dz;
}

/* Back-project pixel (u, v) (Sec. V-B).  Pinhole camera, x right, y down,
 * z forward, pixel centres at +0.5.  FP32, fixed order. */
void or_pixel_ray(const float M[9], const float c[3], float fx, float fy, float cx, float cy,
                  int u, int v, float o[3], float d[3]) {
  float x = (((float)u + 0.5f) - cx) / fx;
  float y = (((float)v + 0.5f) - cy) / fy;
  float dd[3];
  for (int k = 0; k < 3; ++k) dd[k] = (M[3 * k + 0] * x + M[3 * k + 1] * y) + M[3 * k + 2];
  float n = sqrtf((dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]);
  for (int k = 0; k < 3; ++k) {
    d[k] = dd[k] / n;
    o[k] = c[k];
  }
}

/* Ray / 3D box intersection giving the truncation interval (Sec. V-B).
 * The box is [-a, a] in the object frame (a = half size, Eq. 4).  Slab test
 * with NaN-ignoring min/max; the near end is clamped at the camera. */
int or_slab(const float o[3], const float d[3], const float half[3], float* tn, float* tf) {
  float tmin = -INFINITY, tmax = INFINITY;
  for (int k = 0; k < 3; ++k) {
    float inv = 1.0f / d[k];
    float t0 = (-half[k] - o[k]) * inv;
    float t1 = (half[k] - o[k]) * inv;
    tmin = fmaxf(tmin, fminf(t0, t1));
    tmax = fminf(tmax, fmaxf(t0, t1));
  }
  float n = fmaxf(tmin, 0.0f);
  *tn = n;
  *tf = tmax;
  return tmax > n;
}

/* Uniform sampling of N points inside the truncation interval (Sec. V-B, no
 * importance sampling).  Midpoints of N equal steps; delta_i = delta. */
void or_sample_positions(const float o[3], const float d[3], const float half[3], float tn,
                         float tf, int N, float* delta, float* dist, float* pos) {
  float dl = (tf - tn) / (float)N;
  *delta = dl;
  for (int i = 0; i < N; ++i) {
    float di = tn + ((float)i + 0.5f) * dl;
    dist[i] = di;
    for (int k = 0; k < 3; ++k) {
      float x = o[k] + di * d[k];
      float p = (x + half[k]) / (half[k] + half[k]);
      p = fminf(fmaxf(p, 0.0f), 1.0f);
      pos[3 * i + k] = p;
    }
  }
}

/* Multiresolution hash encoding of one point (the encoding of Sec. V, as
 * defined by the cited Mueller et al. 2022).  idx/w: 8 corners per level;
 * e: L*2 features.  Corner b uses bit0 = x, bit1 = y, bit2 = z. */
void or_encode(const or_levels* lv, const float p[3], const double* grid, uint32_t* idx,
               double* w, double* e) {
  for (int l = 0; l < lv->L; ++l) {
    int N = lv->N[l];
    float Nf = (float)N;
    int cell[3];
    float fr[3];
    for (int k = 0; k < 3; ++k) {
      float g = p[k] * Nf;
      int ci = (int)floorf(g);
      if (ci < 0) ci = 0;
      if (ci > N - 1) ci = N - 1;
      cell[k] = ci;
      fr[k] = g - (float)ci;
    }
    const double* G = grid + lv->off[l];
    e[2 * l + 0] = 0.0;
    e[2 * l + 1] = 0.0;
    for (int b = 0; b < 8; ++b) {
      uint32_t vx = (uint32_t)(cell[0] + (b & 1));
      uint32_t vy = (uint32_t)(cell[1] + ((b >> 1) & 1));
      uint32_t vz = (uint32_t)(cell[2] + ((b >> 2) & 1));
      uint32_t id;
      if (lv->hashed[l]) {
        id = (vx * 1u) ^ (vy * 2654435761u) ^ (vz * 805459861u);
        id &= (uint32_t)(lv->T[l] - 1);
      } else {
        uint32_t n1 = (uint32_t)N + 1u;
        id = vx + vy * n1 + vz * n1 * n1;
      }
      double wb = 1.0;
      for (int k = 0; k < 3; ++k) wb *= ((b >> k) & 1) ? (double)fr[k] : 1.0 - (double)fr[k];
      idx[8 * l + b] = id;
      w[8 * l + b] = wb;
      e[2 * l + 0] += wb * G[2 * (int64_t)id + 0];
      e[2 * l + 1] += wb * G[2 * (int64_t)id + 1];
    }
  }
}

/* BF16 mode of the MLP.  The paper does not state its precision; this mode
 * is the precision choice of the GPU path's "BF16 MLP": every operand of an
 * MLP contraction -- the weights, each layer's input, each adjoint entering
 * a contraction, and both factors of every weight-gradient outer product --
 * is rounded to BF16 (IEEE binary32's exponent range with 8 significant
 * bits, round to nearest, ties to even); sums, activations, compositing,
 * the loss and the encoding stay FP64. */
double or_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  if (fabs(x) < 0x1p-126) /* BF16 subnormals: multiples of 2^-133 */
    return ldexp(nearbyint(ldexp(x, 133)), -133);
  /* keep 7 of the 52 stored fraction bits; the dropped 45 bits round to
   * nearest, ties to the even kept value (a carry may move to the next
   * binade, which is the correct result) */
  uint64_t u;
  memcpy(&u, &x, sizeof u);
  const int drop = 45;
  u += (((uint64_t)1 << (drop - 1)) - 1) + ((u >> drop) & 1u);
  u &= ~(((uint64_t)1 << drop) - 1);
  memcpy(&x, &u, sizeof x);
  return x;
}

/* Distance from x to the nearest point where or_bf16 changes its result (a
 * midpoint between two neighbouring BF16 values).  Test infrastructure: a
 * value within rounding error of such a point may round either way. */
double or_bf16_gap(double x) {
  if (x == 0.0 || !isfinite(x)) return INFINITY;
  int ex;
  frexp(x, &ex); /* |x| in [2^(ex-1), 2^ex) */
  int q = ex - 8;
  if (q < -133) q = -133;
  const double s = fabs(ldexp(x, -q)); /* in [128, 256) for normal values */
  return fabs(s - floor(s) - 0.5) * ldexp(1.0, q);
}

/* Tests only: with a nonzero jitter every rounded operand other than a
 * weight is first moved by at most rel |x| (a deterministic function of x),
 * which imitates a computation of it with rounding error; the BF16
 * allowances of the tests must cover the change this makes. */
static double g_bf16_jitter = 0.0;
void or_bf16_set_jitter(double rel) { g_bf16_jitter = rel; }
/* Tests only: with a nonzero tie jitter the backward takes the branch of
 * every ReLU unit from its pre-activation moved by at most rel times the sum
 * of |terms| that form it (a deterministic function of its value), with the
 * forward unchanged: a branch taken the other way, as a computation with
 * rounding error may take it near a tie; the tie allowances of the tests
 * must cover the change this makes.  The seed selects another such function
 * for both jitters. */
static double g_tie_jitter = 0.0;
static uint64_t g_jitter_seed = 0;
void or_set_tie_jitter(double rel) { g_tie_jitter = rel; }
void or_set_jitter_seed(uint64_t seed) { g_jitter_seed = seed; }

/* a deterministic value in [-1, 1) from the bits of x and the seed */
static double jitter_unit(double x) {
  uint64_t u;
  memcpy(&u, &x, sizeof u);
  u += 0x9E3779B97F4A7C15ull * (1ull + 2ull * g_jitter_seed); /* splitmix64 finaliser */
  u = (u ^ (u >> 30)) * 0xBF58476D1CE4E5B9ull;
  u = (u ^ (u >> 27)) * 0x94D049BB133111EBull;
  u ^= u >> 31;
  return (double)(u >> 11) * 0x1p-53 * 2.0 - 1.0;
}

static double jitter(double x) { return x * (1.0 + g_bf16_jitter * jitter_unit(x)); }


/* an operand of a contraction (activation or adjoint) */
static inline double rbf(int on, double x) {
  return on ? or_bf16(g_bf16_jitter != 0.0 ? jitter(x) : x) : x;
}
/* a weight (an FP32 value on either side: never jittered) */
static inline double rbw(int on, double x) { return on ? or_bf16(x) : x; }

/* Branch of a ReLU unit in the backward: its output h is positive; under
 * the tie jitter, its pre-activation (row W of K weights against the layer
 * input x) moved as described above is. */
static int relu_open(int bf, double h, const double* W, const double* x, int K) {
  if (g_tie_jitter == 0.0) return h > 0.0;
  double pre = 0.0, mag = 0.0;
  for (int j = 0; j < K; ++j) {
    const double t = rbw(bf, W[j]) * rbf(bf, x[j]);
    pre += t;
    mag += fabs(t);
  }
  return pre + g_tie_jitter * mag * jitter_unit(pre) > 0.0;
}

/* Density / colour MLP (Sec. V: a single hidden layer of 64 per head; position
 * only, no view direction, Sec. V-B; the model-size study of Table 4 also
 * trains density MLPs of 2 and 3 hidden layers).  h_0 = ReLU(W1 e),
 * h_k = ReLU(Wh_k h_{k-1}) for k < layers, y = W2 h_{layers-1},
 * sigma = exp(min(y0, 15)), h2 = ReLU(W3 y[1..15]), rgb = sigmoid(W4 h2).
 * h1 receives the layers hidden activations, 64 each (unrounded).  With
 * bf16, every weight and every layer input is rounded by or_bf16 where a
 * contraction reads it. */
void or_mlp_forward(int din, int layers, int bf16, const double* mlp, const double* e, double* h1,
                    double* y, double* h2, double* sigma, double* rgb, double* rgbc) {
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (layers - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  const double* W4 = W3 + OR_HIDDEN * OR_GEO;
  for (int i = 0; i < OR_HIDDEN; ++i) {
    double s = 0.0;
    for (int j = 0; j < din; ++j) s += rbw(bf16, W1[i * din + j]) * rbf(bf16, e[j]);
    h1[i] = s > 0.0 ? s : 0.0;
  }
  for (int k = 1; k < layers; ++k) {
    const double* W = Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* hp = h1 + (k - 1) * OR_HIDDEN;
    double* hn = h1 + k * OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i) {
      double s = 0.0;
      for (int j = 0; j < OR_HIDDEN; ++j) s += rbw(bf16, W[i * OR_HIDDEN + j]) * rbf(bf16, hp[j]);
      hn[i] = s > 0.0 ? s : 0.0;
    }
  }
  const double* hl = h1 + (layers - 1) * OR_HIDDEN;
  for (int i = 0; i < OR_DOUT; ++i) {
    double s = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) s += rbw(bf16, W2[i * OR_HIDDEN + j]) * rbf(bf16, hl[j]);
    y[i] = s;
  }
  *sigma = exp(fmin(y[0], 15.0));
  for (int i = 0; i < OR_HIDDEN; ++i) {
    double s = 0.0;
    for (int j = 0; j < OR_GEO; ++j) s += rbw(bf16, W3[i * OR_GEO + j]) * rbf(bf16, y[1 + j]);
    h2[i] = s > 0.0 ? s : 0.0;
  }
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) s += rbw(bf16, W4[i * OR_HIDDEN + j]) * rbf(bf16, h2[j]);
    rgb[i] = 1.0 / (1.0 + exp(-s));
    if (rgbc) rgbc[i] = 1.0 / (1.0 + exp(s)); /* 1 - rgb without cancellation */
  }
}

/* Volume rendering (Sec. V-B, Eq. 6): o_i = 1 - exp(-sigma_i delta_i),
 * w_i = o_i prod_{j<i} (1 - o_j), C = sum w_i c_i, D = sum w_i d_i.
 * Background rays add T_end * C_random (reading of Eq. 9). */
void or_composite(int N, const double* sigma, const double* rgb, const double* dist, double delta,
                  int background, const double crand[3], double C[3], double* D, double* Tend,
                  double* w) {
  double S = 0.0;
  C[0] = C[1] = C[2] = 0.0;
  *D = 0.0;
  for (int i = 0; i < N; ++i) {
    double tau = sigma[i] * delta;
    double T = exp(-S);
    double a = -expm1(-tau);
    double wi = T * a;
    w[i] = wi;
    for (int k = 0; k < 3; ++k) C[k] += wi * rgb[3 * i + k];
    *D += wi * dist[i];
    S += tau;
  }
  *Tend = exp(-S);
  if (background)
    for (int k = 0; k < 3; ++k) C[k] += *Tend * crand[k];
}

/* Candidate pixels of one object in one keyframe: the object's 2D detection
 * box (Sec. V-B back-projects "pixels within the object's detection box"),
 * read as the bounding box of its mask pixels widened by margin_pct percent
 * of its size on every side (integer ceiling), clamped to the image. */
int or_candidate_rect(const int32_t* mask, int W, int H, int instance, int margin_pct,
                      int32_t rect[4]) {
  int xmin = W, xmax = -1, ymin = H, ymax = -1;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      if (mask[(int64_t)y * W + x] == instance) {
        if (x < xmin) xmin = x;
        if (x > xmax) xmax = x;
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
      }
  if (xmax < 0) return 0;
  int w0 = xmax - xmin + 1, h0 = ymax - ymin + 1;
  int mx = (w0 * margin_pct + 99) / 100, my = (h0 * margin_pct + 99) / 100;
  int x0 = xmin - mx < 0 ? 0 : xmin - mx;
  int y0 = ymin - my < 0 ? 0 : ymin - my;
  int x1 = xmax + mx > W - 1 ? W - 1 : xmax + mx;
  int y1 = ymax + my > H - 1 ? H - 1 : ymax + my;
  rect[0] = x0;
  rect[1] = y0;
  rect[2] = x1 - x0 + 1;
  rect[3] = y1 - y0 + 1;
  return 1;
}

/* Draw ray r of step `step` for object `obj` (Sec. VI: rays drawn at random
 * from all training images of the object; Sec. V-B: classified by the
 * instance mask into object rays R_o, background rays R_b and occluder rays).
 * Candidates are enumerated keyframe by keyframe, row-major inside each
 * candidate rectangle; the draw is uniform with replacement. */
void or_draw_ray(const or_config* cfg, int obj, int step, int r, int nkf, const or_keyframe* kfs,
                 int instance, or_ray* out) {
  memset(out, 0, sizeof(*out));
  uint32_t key[2] = {(uint32_t)cfg->seed ^ (uint32_t)obj, (uint32_t)(cfg->seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)step, (uint32_t)r, 0u, 0u};
  uint32_t x[4];
  or_philox4x32_10(ctr, key, x);
  int64_t ncand = 0;
  for (int k = 0; k < nkf; ++k) ncand += (int64_t)kfs[k].w * kfs[k].h;
  int64_t q = (int64_t)(((uint64_t)x[0] * (uint64_t)ncand) >> 32);
  int k = 0;
  while (q >= (int64_t)kfs[k].w * kfs[k].h) {
    q -= (int64_t)kfs[k].w * kfs[k].h;
    ++k;
  }
  const or_keyframe* kf = &kfs[k];
  int u = kf->x0 + (int)(q % kf->w);
  int v = kf->y0 + (int)(q / kf->w);
  out->kf = k;
  out->u = u;
  out->v = v;
  for (int j = 0; j < 3; ++j) out->Crand[j] = (float)(x[j + 1] >> 8) * (1.0f / 16777216.0f);
  int64_t pix = (int64_t)v * kf->W + u;
  int m = kf->mask[pix];
  out->cls = (m == instance) ? 1 : (m == 0 ? 2 : 0);
  for (int j = 0; j < 3; ++j) out->C[j] = (float)kf->rgb[3 * pix + j] / 255.0f;
  out->has_depth = 0;
  out->D = 0.0f;
  if (kf->depth && out->cls == 1) {
    float z = kf->depth[pix];
    if (z > 0.0f && isfinite(z)) {
      /* sparse depth is camera z; the loss compares ray distance (Eq. 8) */
      float xn = (((float)u + 0.5f) - kf->cx) / kf->fx;
      float yn = (((float)v + 0.5f) - kf->cy) / kf->fy;
      out->has_depth = 1;
      out->D = z * sqrtf((xn * xn + yn * yn) + 1.0f);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* One training step of one object: draw, render, loss (Eq. 7-11), gradient
 * of the loss with respect to every parameter.  `grad` (may be NULL) is
 * overwritten with dL/dparams; `grad_abs` (may be NULL) with the magnitude of
 * the same gradient (see sample_backward_magnitude).  `rays` (may be NULL) receives the per-ray
 * record.  The loss is L = (1/B) sum_r l_r. */
typedef struct {
  uint32_t* idx;
  double *w, *e, *h1, *y, *h2, *sigma, *rgb, *rgbc, *dist, *wts, *dsig, *dsig_m, *tnext;
  float *pos, *dist32;
  int* live; /* sample not skipped by the occupancy bitfield */
  struct or_fpert_s* fp; /* tests only: BF16 forward bounds (bf16_ray_allowance) */
  int fp_valid;          /* fp holds the bounds of the current ray */
} or_scratch;

static void scratch_alloc(or_scratch* s, int N, int L, int layers) {
  s->idx = (uint32_t*)malloc(sizeof(uint32_t) * N * L * 8);
  s->w = (double*)malloc(sizeof(double) * N * L * 8);
  s->e = (double*)malloc(sizeof(double) * N * L * 2);
  s->h1 = (double*)malloc(sizeof(double) * N * OR_HIDDEN * layers);
  s->y = (double*)malloc(sizeof(double) * N * OR_DOUT);
  s->h2 = (double*)malloc(sizeof(double) * N * OR_HIDDEN);
  s->sigma = (double*)malloc(sizeof(double) * N);
  s->rgb = (double*)malloc(sizeof(double) * N * 3);
  s->rgbc = (double*)malloc(sizeof(double) * N * 3);
  s->dist = (double*)malloc(sizeof(double) * N);
  s->wts = (double*)malloc(sizeof(double) * N);
  s->dsig = (double*)malloc(sizeof(double) * N);
  s->dsig_m = (double*)malloc(sizeof(double) * N);
  s->tnext = (double*)malloc(sizeof(double) * N);
  s->pos = (float*)malloc(sizeof(float) * N * 3);
  s->dist32 = (float*)malloc(sizeof(float) * N);
  s->live = (int*)malloc(sizeof(int) * N);
  s->fp = NULL; /* allocated on first use (BF16 mode, tests) */
  s->fp_valid = 0;
}

static void scratch_free(or_scratch* s) {
  free(s->idx); free(s->w); free(s->e); free(s->h1); free(s->y); free(s->h2);
  free(s->sigma); free(s->rgb); free(s->rgbc); free(s->dist); free(s->wts); free(s->dsig); free(s->dsig_m); free(s->tnext);
  free(s->pos); free(s->dist32); free(s->live);
  free(s->fp);
}

/* Backward of one sample through the MLPs and the encoding.  dsig, dc are
 * dl/dsigma and dl/dc of this sample; adds into grad (grid, then MLP).  h1
 * holds the hidden activations of the density MLP's lv->mlp_layers layers.
 * In BF16 mode (lv->mlp_bf16) every operand of a contraction is rounded by
 * or_bf16, as in the forward: the weights, the adjoint entering each
 * transposed product, and both factors of each weight-gradient product. */
static void sample_backward(const or_levels* lv, int din, const double* mlp, const uint32_t* idx,
                            const double* w, const double* e, const double* h1, const double* y,
                            const double* h2, double sigma, const double* rgb,
                            const double* rgbc, double dsig, const double* dc, double* grad) {
  const int nh = lv->mlp_layers, bf = lv->mlp_bf16;
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  const double* W4 = W3 + OR_HIDDEN * OR_GEO;
  double* gG = grad;
  double* gW1 = grad + or_grid_params(lv);
  double* gWh = gW1 + OR_HIDDEN * din;
  double* gW2 = gWh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  double* gW3 = gW2 + OR_DOUT * OR_HIDDEN;
  double* gW4 = gW3 + OR_HIDDEN * OR_GEO;
  double dz4[3], dh2[OR_HIDDEN], dy[OR_DOUT], dh[OR_HIDDEN], dp[OR_HIDDEN],
      de[2 * OR_MAX_LEVELS];
  /* sigmoid'(z) = sigmoid(z) sigmoid(-z): rgbc = 1 - rgb formed without cancellation */
  for (int k = 0; k < 3; ++k) dz4[k] = dc[k] * rgb[k] * rgbc[k];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < OR_HIDDEN; ++j) gW4[k * OR_HIDDEN + j] += rbf(bf, dz4[k]) * rbf(bf, h2[j]);
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += rbw(bf, W4[k * OR_HIDDEN + j]) * rbf(bf, dz4[k]);
    dh2[j] = relu_open(bf, h2[j], W3 + j * OR_GEO, y + 1, OR_GEO) ? s : 0.0;
  }
  for (int j = 0; j < OR_HIDDEN; ++j)
    for (int g = 0; g < OR_GEO; ++g) gW3[j * OR_GEO + g] += rbf(bf, dh2[j]) * rbf(bf, y[1 + g]);
  for (int g = 0; g < OR_GEO; ++g) {
    double s = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) s += rbw(bf, W3[j * OR_GEO + g]) * rbf(bf, dh2[j]);
    dy[1 + g] = s;
  }
  dy[0] = y[0] < 15.0 ? dsig * sigma : 0.0;
  /* last hidden layer */
  const double* hl = h1 + (nh - 1) * OR_HIDDEN;
  for (int i = 0; i < OR_DOUT; ++i)
    for (int j = 0; j < OR_HIDDEN; ++j) gW2[i * OR_HIDDEN + j] += rbf(bf, dy[i]) * rbf(bf, hl[j]);
  {
    /* the last hidden layer's rows and input */
    const double* Wl = nh == 1 ? W1 : Wh + (nh - 2) * OR_HIDDEN * OR_HIDDEN;
    const double* xl = nh == 1 ? e : h1 + (nh - 2) * OR_HIDDEN;
    const int Kl = nh == 1 ? din : OR_HIDDEN;
    for (int j = 0; j < OR_HIDDEN; ++j) {
      double s = 0.0;
      for (int i = 0; i < OR_DOUT; ++i) s += rbw(bf, W2[i * OR_HIDDEN + j]) * rbf(bf, dy[i]);
      dh[j] = relu_open(bf, hl[j], Wl + j * Kl, xl, Kl) ? s : 0.0;
    }
  }
  /* hidden-to-hidden layers, last to first: dh is the adjoint of h_k */
  for (int k = nh - 1; k >= 1; --k) {
    const double* W = Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    double* gW = gWh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* hp = h1 + (k - 1) * OR_HIDDEN;
    const double* Wp = k == 1 ? W1 : Wh + (k - 2) * OR_HIDDEN * OR_HIDDEN;
    const double* xp = k == 1 ? e : h1 + (k - 2) * OR_HIDDEN;
    const int Kp = k == 1 ? din : OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i)
      for (int j = 0; j < OR_HIDDEN; ++j) gW[i * OR_HIDDEN + j] += rbf(bf, dh[i]) * rbf(bf, hp[j]);
    for (int j = 0; j < OR_HIDDEN; ++j) {
      double s = 0.0;
      for (int i = 0; i < OR_HIDDEN; ++i) s += rbw(bf, W[i * OR_HIDDEN + j]) * rbf(bf, dh[i]);
      dp[j] = relu_open(bf, hp[j], Wp + j * Kp, xp, Kp) ? s : 0.0;
    }
    memcpy(dh, dp, sizeof(dh));
  }
  for (int j = 0; j < OR_HIDDEN; ++j)
    for (int q = 0; q < din; ++q) gW1[j * din + q] += rbf(bf, dh[j]) * rbf(bf, e[q]);
  for (int q = 0; q < din; ++q) {
    double s = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) s += rbw(bf, W1[j * din + q]) * rbf(bf, dh[j]);
    de[q] = s;
  }
  for (int l = 0; l < lv->L; ++l)
    for (int b = 0; b < 8; ++b) {
      int64_t at = lv->off[l] + 2 * (int64_t)idx[8 * l + b];
      gG[at + 0] += w[8 * l + b] * de[2 * l + 0];
      gG[at + 1] += w[8 * l + b] * de[2 * l + 1];
    }
}

/* The same backward on magnitudes: every weight, activation and upstream
 * adjoint replaced by its absolute value, so each sum becomes a sum of
 * |terms|.  The result bounds, to first order, how far a gradient computed
 * with rounding (in any summation order) can move: rounding error of each
 * operation is relative to these magnitudes, not to the possibly cancelled
 * value.  Test infrastructure for the per-entry tolerance. */
static void sample_backward_magnitude(const or_levels* lv, int din, const double* mlp,
                                      const uint32_t* idx, const double* w, const double* e,
                                      const double* h1, const double* y, const double* h2,
                                      double sigma, const double* rgb, const double* rgbc,
                                      double dsig_m, const double* dc_m, int all_branches,
                                      double* mag) {
  const int nh = lv->mlp_layers, bf = lv->mlp_bf16;
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  const double* W4 = W3 + OR_HIDDEN * OR_GEO;
  double* mG = mag;
  double* mW1 = mag + or_grid_params(lv);
  double* mWh = mW1 + OR_HIDDEN * din;
  double* mW2 = mWh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  double* mW3 = mW2 + OR_DOUT * OR_HIDDEN;
  double* mW4 = mW3 + OR_HIDDEN * OR_GEO;
#define A(x) fabs(rbf(bf, (x)))
  double dz4[3], dh2[OR_HIDDEN], dy[OR_DOUT], dh[OR_HIDDEN], dp[OR_HIDDEN],
      de[2 * OR_MAX_LEVELS];
  for (int k = 0; k < 3; ++k) dz4[k] = dc_m[k] * rgb[k] * rgbc[k];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < OR_HIDDEN; ++j) mW4[k * OR_HIDDEN + j] += A(dz4[k]) * A(h2[j]);
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += A(W4[k * OR_HIDDEN + j]) * A(dz4[k]);
    dh2[j] = (h2[j] > 0.0 || all_branches) ? s : 0.0;
  }
  for (int j = 0; j < OR_HIDDEN; ++j)
    for (int g = 0; g < OR_GEO; ++g) mW3[j * OR_GEO + g] += A(dh2[j]) * A(y[1 + g]);
  for (int g = 0; g < OR_GEO; ++g) {
    double s = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) s += A(W3[j * OR_GEO + g]) * A(dh2[j]);
    dy[1 + g] = s;
  }
  dy[0] = (y[0] < 15.0 || all_branches) ? dsig_m * sigma : 0.0;
  const double* hl = h1 + (nh - 1) * OR_HIDDEN;
  for (int i = 0; i < OR_DOUT; ++i)
    for (int j = 0; j < OR_HIDDEN; ++j) mW2[i * OR_HIDDEN + j] += A(dy[i]) * A(hl[j]);
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double s = 0.0;
    for (int i = 0; i < OR_DOUT; ++i) s += A(W2[i * OR_HIDDEN + j]) * A(dy[i]);
    dh[j] = (hl[j] > 0.0 || all_branches) ? s : 0.0;
  }
  for (int k = nh - 1; k >= 1; --k) {
    const double* W = Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    double* mW = mWh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* hp = h1 + (k - 1) * OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i)
      for (int j = 0; j < OR_HIDDEN; ++j) mW[i * OR_HIDDEN + j] += A(dh[i]) * A(hp[j]);
    for (int j = 0; j < OR_HIDDEN; ++j) {
      double s = 0.0;
      for (int i = 0; i < OR_HIDDEN; ++i) s += A(W[i * OR_HIDDEN + j]) * A(dh[i]);
      dp[j] = (hp[j] > 0.0 || all_branches) ? s : 0.0;
    }
    memcpy(dh, dp, sizeof(dh));
  }
  for (int j = 0; j < OR_HIDDEN; ++j)
    for (int q = 0; q < din; ++q) mW1[j * din + q] += A(dh[j]) * A(e[q]);
  for (int q = 0; q < din; ++q) {
    double s = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) s += A(W1[j * din + q]) * A(dh[j]);
    de[q] = s;
  }
#undef A
  for (int l = 0; l < lv->L; ++l)
    for (int b = 0; b < 8; ++b) {
      int64_t at = lv->off[l] + 2 * (int64_t)idx[8 * l + b];
      mG[at + 0] += w[8 * l + b] * de[2 * l + 0];
      mG[at + 1] += w[8 * l + b] * de[2 * l + 1];
    }
}

/* Occupancy skip (an addition to the paper's method for long ray budgets): a
 * 64^3 bitfield over the object's unit cube, bit x + 64 y + 4096 z of cell
 * (floor(64 p), clamped), least significant bit first in each byte.  A sample
 * in a cell whose bit is 0 has density 0: it adds nothing to the rendering,
 * the density loss or the gradient. */
int or_occupied(const uint8_t* occ, const float p[3]) {
  if (!occ) return 1;
  int c[3];
  for (int k = 0; k < 3; ++k) {
    int ci = (int)floorf(p[k] * 64.0f);
    c[k] = ci < 0 ? 0 : (ci > 63 ? 63 : ci);
  }
  const int bit = c[0] + 64 * c[1] + 4096 * c[2];
  return (occ[bit >> 3] >> (bit & 7)) & 1;
}

/* Forward of one ray with N uniform samples in [tn, tf]: positions, encoding,
 * MLPs (kept in s for the backward), and Eq. 6 (plus T_end C_rand for a
 * background ray). */
static void ray_forward(const or_levels* lv, int N, const double* params, const float o[3],
                        const float d[3], const float half[3], float tn, float tf, float* delta,
                        or_scratch* s, int bg, const double crand[3], double C[3], double* D,
                        double* Tend, const uint8_t* occ) {
  const int L = lv->L, din = 2 * L, nh = lv->mlp_layers;
  const double* mlp = params + or_grid_params(lv);
  or_sample_positions(o, d, half, tn, tf, N, delta, s->dist32, s->pos);
  s->fp_valid = 0;
  for (int i = 0; i < N; ++i) s->dist[i] = (double)s->dist32[i];
  for (int i = 0; i < N; ++i) {
    s->live[i] = or_occupied(occ, s->pos + 3 * i);
    or_encode(lv, s->pos + 3 * i, params, s->idx + 8 * L * i, s->w + 8 * L * i, s->e + 2 * L * i);
    or_mlp_forward(din, nh, lv->mlp_bf16, mlp, s->e + 2 * L * i, s->h1 + OR_HIDDEN * nh * i,
                   s->y + OR_DOUT * i, s->h2 + OR_HIDDEN * i, s->sigma + i, s->rgb + 3 * i,
                   s->rgbc + 3 * i);
    if (!s->live[i]) s->sigma[i] = 0.0;
  }
  or_composite(N, s->sigma, s->rgb, s->dist, (double)*delta, bg, crand, C, D, Tend, s->wts);
}

/* Backward of one ray given dl/dC (gC), dl/dD (gD), dl/dT_end (gT) and the
 * per-sample density-loss weight dens (Eq. 10 term, background rays only).
 * Adjoint of Eq. 6: dC/dtau_i = T_{i+1} c_i - sum_{j>i} w_j c_j, and every
 * tau_i enters T_end = exp(-sum tau) (background rays composite T_end C_rand).
 * Adds dl/dparams into grad and, if mag is not NULL, the magnitude of the same
 * backward into mag, with gCm (may be NULL: |gC|) the magnitude of the terms
 * that form gC (a colour residual's is that of the colour and its target). */
static void ray_backward(const or_levels* lv, int N, const double* params, double delta,
                         or_scratch* s, int bg, const double crand[3], double Tend,
                         const double gC[3], const double* gCm, double gD, double gT, double dens,
                         double* grad, double* mag) {
  const int L = lv->L, din = 2 * L, nh = lv->mlp_layers;
  const double* mlp = params + or_grid_params(lv);
  double gA[3];
  for (int k = 0; k < 3; ++k) gA[k] = gCm ? gCm[k] : fabs(gC[k]);
  double suf_c[3] = {0.0, 0.0, 0.0}, suf_d = 0.0;
  double S_i = 0.0;
  for (int i = 0; i < N; ++i) {
    S_i += s->sigma[i] * delta;
    s->tnext[i] = exp(-S_i);
  }
  const double* Tnext = s->tnext;
  for (int i = N - 1; i >= 0; --i) {
    double a = 0.0, am = 0.0;
    for (int k = 0; k < 3; ++k) a += gC[k] * (Tnext[i] * s->rgb[3 * i + k] - suf_c[k]);
    if (bg)
      for (int k = 0; k < 3; ++k) a -= gC[k] * Tend * crand[k];
    a += gD * (Tnext[i] * s->dist[i] - suf_d);
    a -= gT * Tend;
    s->dsig[i] = s->live[i] ? a * delta + dens : 0.0;
    /* magnitude of the same adjoint (for the tolerance of the tests) */
    for (int k = 0; k < 3; ++k) am += gA[k] * (Tnext[i] * s->rgb[3 * i + k] + suf_c[k]);
    if (bg)
      for (int k = 0; k < 3; ++k) am += gA[k] * Tend * crand[k];
    am += fabs(gD) * (Tnext[i] * s->dist[i] + suf_d) + fabs(gT) * Tend;
    s->dsig_m[i] = s->live[i] ? am * delta + dens : 0.0;
    for (int k = 0; k < 3; ++k) suf_c[k] += s->wts[i] * s->rgb[3 * i + k];
    suf_d += s->wts[i] * s->dist[i];
  }
  for (int i = 0; i < N; ++i) {
    if (!s->live[i]) continue; /* density 0 by construction: no dependence on parameters */
    double dci[3];
    for (int k = 0; k < 3; ++k) dci[k] = s->wts[i] * gC[k];
    sample_backward(lv, din, mlp, s->idx + 8 * L * i, s->w + 8 * L * i, s->e + 2 * L * i,
                    s->h1 + OR_HIDDEN * nh * i, s->y + OR_DOUT * i, s->h2 + OR_HIDDEN * i,
                    s->sigma[i], s->rgb + 3 * i, s->rgbc + 3 * i, s->dsig[i], dci, grad);
    if (mag) {
      for (int k = 0; k < 3; ++k) dci[k] = s->wts[i] * gA[k];
      sample_backward_magnitude(lv, din, mlp, s->idx + 8 * L * i, s->w + 8 * L * i,
                                s->e + 2 * L * i, s->h1 + OR_HIDDEN * nh * i,
                                s->y + OR_DOUT * i, s->h2 + OR_HIDDEN * i, s->sigma[i],
                                s->rgb + 3 * i, s->rgbc + 3 * i, s->dsig_m[i], dci, 0, mag);
    }
  }
}

/* Test infrastructure.  A gradient entry is not unique when it depends on a
 * discrete decision (a ReLU branch, the density clamp, the sign of the depth
 * error) that a computation with rounding error could take the other way.
 * The relative distance of a decision from its tie is |pre-activation| over
 * the sum of |terms| that form it; sample_ties returns the smallest one over
 * the sample's decisions.  In BF16 mode the pre-activations are formed from
 * the rounded operands, and F (may be NULL) holds how far the BF16 decisions
 * upstream can move each pre-activation: that distance is taken off. */
struct or_fpert_s;
static double sample_ties(const or_levels* lv, const double* mlp, const double* e,
                          const double* h1, const double* y, const struct or_fpert_s* F);
/* ---- BF16 rounding decisions (test infrastructure) ------------------------
 * In BF16 mode each rounded operand is a discrete decision.  The GPU forms
 * the value in FP32, the oracle in FP64: a value within FP32 rounding error
 * of a BF16 midpoint may round to either neighbour, and both results are
 * correct.  The functions below bound, per gradient entry, how far the
 * other choices can move the result.  Each value x carries a bound P_x of
 * how far such choices upstream can move it; its rounding can flip when
 * its distance to the nearest midpoint is at most P_x + OR_KBF16 s_x, with
 * s_x the error scale of its own FP32 computation (the sum of |terms| that
 * form it: exact BF16 products, so only the FP32 sum rounds, at most about
 * 64 FP32 units of s_x for a 64-term sum in any order), and a flip adds one
 * BF16 unit in the last place to P.  Bounds combine as
 * P(a b) <= |a| P_b + P_a |b| + P_a P_b and P(sum) <= sum P (rigorous for
 * the products and sums; first order through exp and the sigmoid). */
#define OR_KBF16 4e-6

/* one BF16 unit in the last place at x (the spacing of BF16 values there) */
static double bf16_ulp(double x) {
  if (x == 0.0 || !isfinite(x)) return 0.0;
  int ex;
  frexp(x, &ex);
  int q = ex - 8;
  if (q < -133) q = -133;
  return ldexp(1.0, q);
}

/* perturbation bound of the rounded value of x, given the bound Px of x */
static double bf16_pert(double x, double Px, double scale) {
  return Px + (or_bf16_gap(x) <= Px + OR_KBF16 * scale ? bf16_ulp(x) : 0.0);
}

typedef struct or_fpert_s {   /* perturbation bounds of one sample's forward */
  double Pe[2 * OR_MAX_LEVELS];              /* rounded encodings */
  double Ppre[OR_HIDDEN * OR_MAX_MLP_LAYERS]; /* hidden pre-activations */
  double Ph[OR_HIDDEN * OR_MAX_MLP_LAYERS];   /* rounded hidden activations */
  double Py[OR_DOUT];                         /* y (unrounded) */
  double Pyr[OR_DOUT];                        /* rounded y */
  double Ppre2[OR_HIDDEN], Ph2[OR_HIDDEN];    /* colour head */
  double Pz[3];                               /* colour logits */
} or_fpert;

static double sample_ties(const or_levels* lv, const double* mlp, const double* e,
                          const double* h1, const double* y, const struct or_fpert_s* F) {
  const int din = 2 * lv->L, nh = lv->mlp_layers, bf = lv->mlp_bf16;
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  double m = INFINITY;
  for (int k = 0; k < nh; ++k) {
    const double* W = k == 0 ? W1 : Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* x = k == 0 ? e : h1 + (k - 1) * OR_HIDDEN;
    const int K = k == 0 ? din : OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i) {
      double pre = 0.0, mag = 0.0;
      for (int j = 0; j < K; ++j) {
        const double t = rbw(bf, W[i * K + j]) * rbf(bf, x[j]);
        pre += t;
        mag += fabs(t);
      }
      const double P = F ? F->Ppre[k * OR_HIDDEN + i] : 0.0;
      if (mag > 0.0) m = fmin(m, (fabs(pre) - P) / mag);
    }
  }
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double pre = 0.0, mag = 0.0;
    for (int g = 0; g < OR_GEO; ++g) {
      const double t = rbw(bf, W3[j * OR_GEO + g]) * rbf(bf, y[1 + g]);
      pre += t;
      mag += fabs(t);
    }
    const double P = F ? F->Ppre2[j] : 0.0;
    if (mag > 0.0) m = fmin(m, (fabs(pre) - P) / mag);
  }
  const double* hl = h1 + (nh - 1) * OR_HIDDEN;
  double mag0 = 0.0;
  for (int j = 0; j < OR_HIDDEN; ++j) mag0 += fabs(rbw(bf, W2[j]) * rbf(bf, hl[j]));
  const double P0 = F ? F->Py[0] : 0.0;
  if (mag0 > 0.0) m = fmin(m, (fabs(y[0] - 15.0) - P0) / mag0);
  return m;
}

static void bf16_forward_pert(const or_levels* lv, const double* grid, const double* mlp,
                              const uint32_t* idx, const double* w, const double* e,
                              const double* h1, const double* y, const double* h2, or_fpert* F) {
  const int L = lv->L, din = 2 * L, nh = lv->mlp_layers, bf = lv->mlp_bf16;
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  const double* W4 = W3 + OR_HIDDEN * OR_GEO;
  for (int l = 0; l < L; ++l)
    for (int j = 0; j < 2; ++j) {
      double sc = 0.0;
      for (int b = 0; b < 8; ++b)
        sc += w[8 * l + b] * fabs(grid[lv->off[l] + 2 * (int64_t)idx[8 * l + b] + j]);
      F->Pe[2 * l + j] = bf16_pert(e[2 * l + j], 0.0, sc);
    }
  for (int i = 0; i < OR_HIDDEN; ++i) {
    double sc = 0.0, p = 0.0;
    for (int q = 0; q < din; ++q) {
      const double wr = fabs(rbw(bf, W1[i * din + q]));
      sc += wr * fabs(rbf(bf, e[q]));
      p += wr * F->Pe[q];
    }
    F->Ppre[i] = p;
    F->Ph[i] = h1[i] > 0.0 ? bf16_pert(h1[i], p, sc) : 0.0;
  }
  for (int k = 1; k < nh; ++k) {
    const double* W = Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* hp = h1 + (k - 1) * OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i) {
      double sc = 0.0, p = 0.0;
      for (int j = 0; j < OR_HIDDEN; ++j) {
        const double wr = fabs(rbw(bf, W[i * OR_HIDDEN + j]));
        sc += wr * fabs(rbf(bf, hp[j]));
        p += wr * F->Ph[(k - 1) * OR_HIDDEN + j];
      }
      F->Ppre[k * OR_HIDDEN + i] = p;
      const double hv = h1[k * OR_HIDDEN + i];
      F->Ph[k * OR_HIDDEN + i] = hv > 0.0 ? bf16_pert(hv, p, sc) : 0.0;
    }
  }
  const double* hl = h1 + (nh - 1) * OR_HIDDEN;
  const double* Pl = F->Ph + (nh - 1) * OR_HIDDEN;
  for (int i = 0; i < OR_DOUT; ++i) {
    double sc = 0.0, p = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) {
      const double wr = fabs(rbw(bf, W2[i * OR_HIDDEN + j]));
      sc += wr * fabs(rbf(bf, hl[j]));
      p += wr * Pl[j];
    }
    F->Py[i] = p;
    F->Pyr[i] = i > 0 ? bf16_pert(y[i], p, sc) : p; /* y0 enters no contraction */
  }
  for (int i = 0; i < OR_HIDDEN; ++i) {
    double sc = 0.0, p = 0.0;
    for (int g = 0; g < OR_GEO; ++g) {
      const double wr = fabs(rbw(bf, W3[i * OR_GEO + g]));
      sc += wr * fabs(rbf(bf, y[1 + g]));
      p += wr * F->Pyr[1 + g];
    }
    F->Ppre2[i] = p;
    F->Ph2[i] = h2[i] > 0.0 ? bf16_pert(h2[i], p, sc) : 0.0;
  }
  for (int k = 0; k < 3; ++k) {
    double p = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) p += fabs(rbw(bf, W4[k * OR_HIDDEN + j])) * F->Ph2[j];
    F->Pz[k] = p;
  }
}

static inline double pprod(double a, double Pa, double b, double Pb) {
  return fabs(a) * Pb + Pa * fabs(b) + Pa * Pb;
}

/* Adds into amb the bound of the change of one sample's gradient
 * contributions, given its forward perturbations F, the bounds dsigma and
 * dcol of its density and colours, the bounds Pdsig and Pdc of its upstream
 * adjoints, and the error scales sc_dz, sc_dy0 of the FP32 colour-logit and
 * density-logit adjoints.  Mirrors sample_backward on (value, bound) pairs. */
static void bf16_backward_pert(const or_levels* lv, const double* mlp, const uint32_t* idx,
                               const double* w, const double* e, const double* h1,
                               const double* y, const double* h2, double sigma, double dsigma,
                               const double* rgb, const double* rgbc, const double dcol[3],
                               double dsig, double Pdsig,
                               const double dc[3], const double Pdc[3], const double sc_dz[3],
                               double sc_dy0, const or_fpert* F, double* amb) {
  const int din = 2 * lv->L, nh = lv->mlp_layers, bf = lv->mlp_bf16;
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  const double* W4 = W3 + OR_HIDDEN * OR_GEO;
  double* aG = amb;
  double* aW1 = amb + or_grid_params(lv);
  double* aWh = aW1 + OR_HIDDEN * din;
  double* aW2 = aWh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  double* aW3 = aW2 + OR_DOUT * OR_HIDDEN;
  double* aW4 = aW3 + OR_HIDDEN * OR_GEO;
  double dz[3], Pdz[3], dh2[OR_HIDDEN], Pdh2[OR_HIDDEN], dy[OR_DOUT], Pdy[OR_DOUT],
      dh[OR_HIDDEN], Pdh[OR_HIDDEN], dp[OR_HIDDEN], Pdp[OR_HIDDEN], Pde[2 * OR_MAX_LEVELS];
  for (int k = 0; k < 3; ++k) {
    const double g = rgb[k] * rgbc[k];
    const double Pg = fabs(1.0 - 2.0 * rgb[k]) * dcol[k] + dcol[k] * dcol[k];
    dz[k] = dc[k] * g;
    Pdz[k] = bf16_pert(dz[k], pprod(dc[k], Pdc[k], g, Pg), sc_dz[k]);
  }
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < OR_HIDDEN; ++j)
      aW4[k * OR_HIDDEN + j] += pprod(rbf(bf, dz[k]), Pdz[k], rbf(bf, h2[j]), F->Ph2[j]);
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double s = 0.0, p = 0.0, sc = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double wr = rbw(bf, W4[k * OR_HIDDEN + j]);
      s += wr * rbf(bf, dz[k]);
      sc += fabs(wr * rbf(bf, dz[k]));
      p += fabs(wr) * Pdz[k];
    }
    dh2[j] = h2[j] > 0.0 ? s : 0.0;
    Pdh2[j] = h2[j] > 0.0 ? bf16_pert(dh2[j], p, sc) : 0.0;
  }
  for (int j = 0; j < OR_HIDDEN; ++j)
    for (int g = 0; g < OR_GEO; ++g)
      aW3[j * OR_GEO + g] += pprod(rbf(bf, dh2[j]), Pdh2[j], rbf(bf, y[1 + g]), F->Pyr[1 + g]);
  for (int g = 0; g < OR_GEO; ++g) {
    double s = 0.0, p = 0.0, sc = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) {
      const double wr = rbw(bf, W3[j * OR_GEO + g]);
      s += wr * rbf(bf, dh2[j]);
      sc += fabs(wr * rbf(bf, dh2[j]));
      p += fabs(wr) * Pdh2[j];
    }
    dy[1 + g] = s;
    Pdy[1 + g] = bf16_pert(s, p, sc);
  }
  dy[0] = y[0] < 15.0 ? dsig * sigma : 0.0;
  Pdy[0] = y[0] < 15.0 ? bf16_pert(dy[0], pprod(dsig, Pdsig, sigma, dsigma), sc_dy0) : 0.0;
  const double* hl = h1 + (nh - 1) * OR_HIDDEN;
  const double* Phl = F->Ph + (nh - 1) * OR_HIDDEN;
  for (int i = 0; i < OR_DOUT; ++i)
    for (int j = 0; j < OR_HIDDEN; ++j)
      aW2[i * OR_HIDDEN + j] += pprod(rbf(bf, dy[i]), Pdy[i], rbf(bf, hl[j]), Phl[j]);
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double s = 0.0, p = 0.0, sc = 0.0;
    for (int i = 0; i < OR_DOUT; ++i) {
      const double wr = rbw(bf, W2[i * OR_HIDDEN + j]);
      s += wr * rbf(bf, dy[i]);
      sc += fabs(wr * rbf(bf, dy[i]));
      p += fabs(wr) * Pdy[i];
    }
    dh[j] = hl[j] > 0.0 ? s : 0.0;
    Pdh[j] = hl[j] > 0.0 ? bf16_pert(dh[j], p, sc) : 0.0;
  }
  for (int k = nh - 1; k >= 1; --k) {
    const double* W = Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    double* aW = aWh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* hp = h1 + (k - 1) * OR_HIDDEN;
    const double* Php = F->Ph + (k - 1) * OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i)
      for (int j = 0; j < OR_HIDDEN; ++j)
        aW[i * OR_HIDDEN + j] += pprod(rbf(bf, dh[i]), Pdh[i], rbf(bf, hp[j]), Php[j]);
    for (int j = 0; j < OR_HIDDEN; ++j) {
      double s = 0.0, p = 0.0, sc = 0.0;
      for (int i = 0; i < OR_HIDDEN; ++i) {
        const double wr = rbw(bf, W[i * OR_HIDDEN + j]);
        s += wr * rbf(bf, dh[i]);
        sc += fabs(wr * rbf(bf, dh[i]));
        p += fabs(wr) * Pdh[i];
      }
      dp[j] = hp[j] > 0.0 ? s : 0.0;
      Pdp[j] = hp[j] > 0.0 ? bf16_pert(dp[j], p, sc) : 0.0;
    }
    memcpy(dh, dp, sizeof(dh));
    memcpy(Pdh, Pdp, sizeof(Pdh));
  }
  for (int j = 0; j < OR_HIDDEN; ++j)
    for (int q = 0; q < din; ++q)
      aW1[j * din + q] += pprod(rbf(bf, dh[j]), Pdh[j], rbf(bf, e[q]), F->Pe[q]);
  for (int q = 0; q < din; ++q) {
    double p = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) p += fabs(rbw(bf, W1[j * din + q])) * Pdh[j];
    Pde[q] = p;
  }
  for (int l = 0; l < lv->L; ++l)
    for (int b = 0; b < 8; ++b) {
      int64_t at = lv->off[l] + 2 * (int64_t)idx[8 * l + b];
      aG[at + 0] += w[8 * l + b] * Pde[2 * l + 0];
      aG[at + 1] += w[8 * l + b] * Pde[2 * l + 1];
    }
}

/* What one ray's BF16 decisions can move (tests only).  Needs ray_forward
 * and (for amb) ray_backward of the ray.  lossmode: gC came from the colour
 * residual (its FP32 error then enters the adjoints' error scales, and its
 * change follows the residual's); otherwise gC, gD, gT were given.  Writes
 * the bounds of the change of the ray's colour (dC), depth (dD), T_end (dT)
 * and summed density (dS) under any choice of the ambiguous roundings, the
 * forward bounds of each sample into s->fp (for the widened ties), and adds
 * into amb (may be NULL) the bound of the change of every gradient entry. */
static void bf16_ray_allowance(const or_levels* lv, int N, const double* params, or_scratch* s,
                               double delta, int bg, const double crand[3], double Tend,
                               const double gC[3], double gD, double gT, int lossmode,
                               const double target[3], double invB, double* amb, double dC[3],
                               double* dD, double* dT, double* dS) {
  const int L = lv->L, nh = lv->mlp_layers;
  const double* mlp = params + or_grid_params(lv);
  double Sx[N + 1], suf[N][3], dsg[N], dcl[N][3];
  Sx[0] = 0.0;
  for (int i = 0; i < N; ++i) Sx[i + 1] = Sx[i] + s->sigma[i] * delta;
  {
    double sc[3] = {0.0, 0.0, 0.0};
    for (int i = N - 1; i >= 0; --i) {
      for (int k = 0; k < 3; ++k) suf[i][k] = sc[k];
      for (int k = 0; k < 3; ++k) sc[k] += s->wts[i] * fabs(s->rgb[3 * i + k]);
    }
  }
  double bgt[3];
  for (int k = 0; k < 3; ++k) bgt[k] = bg ? Tend * crand[k] : 0.0;
  /* forward: bounds of each sample's density and colours */
  if (!s->fp) s->fp = (or_fpert*)calloc((size_t)N, sizeof(or_fpert));
  s->fp_valid = 1;
  double sum_ds = 0.0;
  for (int i = 0; i < N; ++i) {
    dsg[i] = 0.0;
    dcl[i][0] = dcl[i][1] = dcl[i][2] = 0.0;
    if (!s->live[i]) continue;
    or_fpert* F = s->fp + i;
    bf16_forward_pert(lv, params, mlp, s->idx + 8 * L * i, s->w + 8 * L * i, s->e + 2 * L * i,
                      s->h1 + OR_HIDDEN * nh * i, s->y + OR_DOUT * i, s->h2 + OR_HIDDEN * i, F);
    dsg[i] = s->sigma[i] * expm1(F->Py[0]);
    for (int k = 0; k < 3; ++k) {
      const double c = s->rgb[3 * i + k];
      dcl[i][k] = fmin(1.0, c * s->rgbc[3 * i + k] * expm1(F->Pz[k]));
    }
    sum_ds += dsg[i];
  }
  /* the ray: transmittances (relative), weights, colour, depth */
  const double rhoT = expm1(delta * sum_ds);
  double dw[N];
  for (int k = 0; k < 3; ++k) dC[k] = bg ? Tend * rhoT * crand[k] : 0.0;
  *dD = 0.0;
  for (int i = 0; i < N; ++i) {
    const double tau = s->sigma[i] * delta;
    dw[i] = s->wts[i] * rhoT + exp(-Sx[i]) * (1.0 + rhoT) * exp(-tau) * expm1(delta * dsg[i]);
    for (int k = 0; k < 3; ++k)
      dC[k] += dw[i] * fabs(s->rgb[3 * i + k]) + (s->wts[i] + dw[i]) * dcl[i][k];
    *dD += dw[i] * s->dist[i];
  }
  *dT = Tend * rhoT;
  *dS = sum_ds;
  if (!amb) return;
  double eg[3] = {0.0, 0.0, 0.0}, dgC[3];
  for (int k = 0; k < 3; ++k) {
    if (lossmode) {
      /* FP32 error scale of the residual, hence of gC (a weight carries the
       * error of its transmittance, relative (1 + S) times the scale) */
      double t = fabs(target[k]) + bgt[k] * (1.0 + Sx[N]);
      for (int i = 0; i < N; ++i) t += s->wts[i] * fabs(s->rgb[3 * i + k]) * (1.0 + Sx[i + 1]);
      eg[k] = 2.0 * invB * t;
    }
    dgC[k] = lossmode ? 2.0 * invB * dC[k] : 0.0;
  }
  for (int i = 0; i < N; ++i) {
    if (!s->live[i]) continue;
    const double Tn = exp(-Sx[i + 1]);
    const double* rgb = s->rgb + 3 * i;
    double dc[3], Pdc[3], sc_dz[3];
    double Pds = fabs(gD) * (Tn * rhoT * s->dist[i] + *dD) + fabs(gT) * *dT;
    double sc_dy0 = s->dsig_m[i] * (1.0 + Sx[i + 1]);
    for (int k = 0; k < 3; ++k) {
      dc[k] = s->wts[i] * gC[k];
      Pdc[k] = pprod(s->wts[i], dw[i], gC[k], dgC[k]);
      sc_dz[k] = fabs(dc[k] * rgb[k] * s->rgbc[3 * i + k]) * (1.0 + Sx[i + 1]) +
                 s->wts[i] * rgb[k] * s->rgbc[3 * i + k] * eg[k];
      const double base = Tn * fabs(rgb[k]) + suf[i][k] + bgt[k];
      Pds += fabs(dgC[k]) * base + fabs(gC[k]) * (Tn * rhoT * fabs(rgb[k]) + Tn * dcl[i][k] +
                                                   dC[k] + (bg ? *dT * crand[k] : 0.0));
      sc_dy0 += delta * base * eg[k];
    }
    Pds *= delta;
    sc_dy0 *= s->sigma[i];
    bf16_backward_pert(lv, mlp, s->idx + 8 * L * i, s->w + 8 * L * i, s->e + 2 * L * i,
                       s->h1 + OR_HIDDEN * nh * i, s->y + OR_DOUT * i, s->h2 + OR_HIDDEN * i,
                       s->sigma[i], dsg[i], rgb, s->rgbc + 3 * i, dcl[i], s->dsig[i], Pds, dc, Pdc,
                       sc_dz, sc_dy0, s->fp + i, amb);
  }
}

/* Tests only.  Adds into amb the change of one sample's gradient
 * contributions when one of its decisions goes the other way.  The decision's
 * pre-activation lies within rounding distance of its tie, so to first order
 * the forward values stay and only the branch of one adjoint changes: the
 * unmasked adjoint v of that unit is added or removed there, and carried
 * down through the layers below with their own decisions; |each term| is
 * added.  stage: 0 .. layers-1 a hidden layer of the density MLP, layers the
 * colour head's hidden layer, layers + 1 the density clamp (unit unused). */
static void flip_delta(const or_levels* lv, int din, const double* mlp, const uint32_t* idx,
                       const double* w, const double* e, const double* h1, const double* y,
                       int stage, int unit, double v, double* amb) {
  const int nh = lv->mlp_layers, bf = lv->mlp_bf16;
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  double* aG = amb;
  double* aW1 = amb + or_grid_params(lv);
  double* aWh = aW1 + OR_HIDDEN * din;
  double* aW2 = aWh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  double* aW3 = aW2 + OR_DOUT * OR_HIDDEN;
  double dy[OR_DOUT], dh[OR_HIDDEN], dp[OR_HIDDEN], de[2 * OR_MAX_LEVELS];
  int k;
  if (stage >= nh) {
    for (int i = 0; i < OR_DOUT; ++i) dy[i] = 0.0;
    if (stage == nh) { /* colour head hidden unit */
      for (int g = 0; g < OR_GEO; ++g) {
        aW3[unit * OR_GEO + g] += fabs(v * rbf(bf, y[1 + g]));
        dy[1 + g] = rbw(bf, W3[unit * OR_GEO + g]) * v;
      }
    } else {
      dy[0] = v;
    }
    const double* hl = h1 + (nh - 1) * OR_HIDDEN;
    for (int i = 0; i < OR_DOUT; ++i)
      if (dy[i] != 0.0)
        for (int j = 0; j < OR_HIDDEN; ++j) aW2[i * OR_HIDDEN + j] += fabs(dy[i] * rbf(bf, hl[j]));
    for (int j = 0; j < OR_HIDDEN; ++j) {
      double t = 0.0;
      for (int i = 0; i < OR_DOUT; ++i) t += rbw(bf, W2[i * OR_HIDDEN + j]) * dy[i];
      dh[j] = hl[j] > 0.0 ? t : 0.0;
    }
    k = nh - 1;
  } else {
    for (int j = 0; j < OR_HIDDEN; ++j) dh[j] = 0.0;
    dh[unit] = v;
    k = stage;
  }
  for (; k >= 1; --k) {
    const double* W = Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    double* aW = aWh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* hp = h1 + (k - 1) * OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i)
      if (dh[i] != 0.0)
        for (int j = 0; j < OR_HIDDEN; ++j) aW[i * OR_HIDDEN + j] += fabs(dh[i] * rbf(bf, hp[j]));
    for (int j = 0; j < OR_HIDDEN; ++j) {
      double t = 0.0;
      for (int i = 0; i < OR_HIDDEN; ++i) t += rbw(bf, W[i * OR_HIDDEN + j]) * dh[i];
      dp[j] = hp[j] > 0.0 ? t : 0.0;
    }
    memcpy(dh, dp, sizeof(dh));
  }
  for (int j = 0; j < OR_HIDDEN; ++j)
    if (dh[j] != 0.0)
      for (int q = 0; q < din; ++q) aW1[j * din + q] += fabs(dh[j] * rbf(bf, e[q]));
  for (int q = 0; q < din; ++q) {
    double t = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) t += rbw(bf, W1[j * din + q]) * dh[j];
    de[q] = t;
  }
  for (int l = 0; l < lv->L; ++l)
    for (int b = 0; b < 8; ++b) {
      const int64_t at = lv->off[l] + 2 * (int64_t)idx[8 * l + b];
      aG[at + 0] += fabs(w[8 * l + b] * de[2 * l + 0]);
      aG[at + 1] += fabs(w[8 * l + b] * de[2 * l + 1]);
    }
}

/* Tests only.  For every decision of one sample that lies closer than kTie
 * (relative to the sum of |terms| that form its pre-activation, less the
 * bound F of what BF16 decisions upstream can move it; F may be NULL) to its
 * tie, adds the change of the sample's contributions under the other branch
 * (flip_delta).  dsig, dc: the sample's signed adjoints of density and
 * colour, as in sample_backward. */
static void sample_tie_deltas(const or_levels* lv, int din, const double* mlp,
                              const uint32_t* idx, const double* w, const double* e,
                              const double* h1, const double* y, const double* h2, double sigma,
                              const double* rgb, const double* rgbc, double dsig,
                              const double* dc, const struct or_fpert_s* F, double kTie,
                              double* amb) {
  const int nh = lv->mlp_layers, bf = lv->mlp_bf16;
  const double* W1 = mlp;
  const double* Wh = W1 + OR_HIDDEN * din;
  const double* W2 = Wh + (nh - 1) * OR_HIDDEN * OR_HIDDEN;
  const double* W3 = W2 + OR_DOUT * OR_HIDDEN;
  const double* W4 = W3 + OR_HIDDEN * OR_GEO;
  double dz4[3], dh2[OR_HIDDEN], dy[OR_DOUT], un[OR_HIDDEN], dh[OR_HIDDEN];
  for (int k = 0; k < 3; ++k) dz4[k] = dc[k] * rgb[k] * rgbc[k];
  /* colour head: unmasked adjoints of its hidden units, and their ties */
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double t = 0.0;
    for (int k = 0; k < 3; ++k) t += rbw(bf, W4[k * OR_HIDDEN + j]) * rbf(bf, dz4[k]);
    double pre = 0.0, mag = 0.0;
    for (int g = 0; g < OR_GEO; ++g) {
      const double q = rbw(bf, W3[j * OR_GEO + g]) * rbf(bf, y[1 + g]);
      pre += q;
      mag += fabs(q);
    }
    const double P = F ? F->Ppre2[j] : 0.0;
    if (mag > 0.0 && (fabs(pre) - P) / mag < kTie)
      flip_delta(lv, din, mlp, idx, w, e, h1, y, nh, j, rbf(bf, t), amb);
    dh2[j] = h2[j] > 0.0 ? t : 0.0;
  }
  for (int g = 0; g < OR_GEO; ++g) {
    double t = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) t += rbw(bf, W3[j * OR_GEO + g]) * rbf(bf, dh2[j]);
    dy[1 + g] = t;
  }
  /* density clamp */
  const double* hl = h1 + (nh - 1) * OR_HIDDEN;
  {
    double mag0 = 0.0;
    for (int j = 0; j < OR_HIDDEN; ++j) mag0 += fabs(rbw(bf, W2[j]) * rbf(bf, hl[j]));
    const double P0 = F ? F->Py[0] : 0.0;
    if (mag0 > 0.0 && (fabs(y[0] - 15.0) - P0) / mag0 < kTie)
      flip_delta(lv, din, mlp, idx, w, e, h1, y, nh + 1, 0, rbf(bf, dsig * sigma), amb);
  }
  dy[0] = y[0] < 15.0 ? dsig * sigma : 0.0;
  /* density MLP, last hidden layer first: un = unmasked adjoint of h_k */
  for (int j = 0; j < OR_HIDDEN; ++j) {
    double t = 0.0;
    for (int i = 0; i < OR_DOUT; ++i) t += rbw(bf, W2[i * OR_HIDDEN + j]) * rbf(bf, dy[i]);
    un[j] = t;
  }
  for (int k = nh - 1; k >= 0; --k) {
    const double* W = k == 0 ? W1 : Wh + (k - 1) * OR_HIDDEN * OR_HIDDEN;
    const double* x = k == 0 ? e : h1 + (k - 1) * OR_HIDDEN;
    const double* hk = h1 + k * OR_HIDDEN;
    const int K = k == 0 ? din : OR_HIDDEN;
    for (int i = 0; i < OR_HIDDEN; ++i) {
      double pre = 0.0, mag = 0.0;
      for (int j = 0; j < K; ++j) {
        const double q = rbw(bf, W[i * K + j]) * rbf(bf, x[j]);
        pre += q;
        mag += fabs(q);
      }
      const double P = F ? F->Ppre[k * OR_HIDDEN + i] : 0.0;
      if (mag > 0.0 && (fabs(pre) - P) / mag < kTie)
        flip_delta(lv, din, mlp, idx, w, e, h1, y, k, i, rbf(bf, un[i]), amb);
      dh[i] = hk[i] > 0.0 ? un[i] : 0.0;
    }
    if (k >= 1) {
      for (int j = 0; j < OR_HIDDEN; ++j) {
        double t = 0.0;
        for (int i = 0; i < OR_HIDDEN; ++i) t += rbw(bf, W[i * OR_HIDDEN + j]) * rbf(bf, dh[i]);
        un[j] = t;
      }
    }
  }
}

/* Tests only.  Smallest distance of a ray's decisions from their ties
 * (dtie: that of its depth-error sign), and into amb (may be NULL) what
 * another choice of each decision closer than 1e-5 to its tie can change:
 * for the ReLU branches and the density clamp of a sample, the change of its
 * contributions under the other branch (sample_tie_deltas); when the ray's
 * depth-error sign ties, twice the magnitude of every sample's contributions
 * with every branch taken.  gC: the ray's colour adjoint.  Needs the forward
 * and ray_backward of the ray (in BF16 mode also bf16_ray_allowance: a
 * pre-activation that BF16 decisions upstream can move by P ties when
 * |pre| <= 1e-5 magnitude + P). */
static double tie_allowance(const or_levels* lv, int N, const double* params, or_scratch* s,
                            const double gC[3], double dtie, double* amb, double* bam) {
  const double kTie = 1e-5;
  const int L = lv->L, nh = lv->mlp_layers;
  const double* mlp = params + or_grid_params(lv);
  double rm = dtie;
  for (int i = 0; i < N; ++i) {
    if (!s->live[i]) continue;
    const struct or_fpert_s* F = lv->mlp_bf16 && s->fp_valid ? s->fp + i : NULL;
    const double sm = sample_ties(lv, mlp, s->e + 2 * L * i, s->h1 + OR_HIDDEN * nh * i,
                                  s->y + OR_DOUT * i, F);
    rm = fmin(rm, sm);
    if (!amb) continue;
    if (dtie < kTie) {
      double dcm[3];
      for (int k = 0; k < 3; ++k) dcm[k] = s->wts[i] * fabs(gC[k]);
      for (int rep = 0; rep < 2; ++rep)
        sample_backward_magnitude(lv, 2 * L, mlp, s->idx + 8 * L * i, s->w + 8 * L * i,
                                  s->e + 2 * L * i, s->h1 + OR_HIDDEN * nh * i,
                                  s->y + OR_DOUT * i, s->h2 + OR_HIDDEN * i, s->sigma[i],
                                  s->rgb + 3 * i, s->rgbc + 3 * i, s->dsig_m[i], dcm, 1, amb);
    }
    if (sm < kTie && bam && lv->mlp_bf16) {
      /* BF16 mode: the other branch also moves the BF16 roundings of the
       * adjoints below the tied unit, each by at most one BF16 unit (2^-8 of
       * the value): within 2^-6 of the sample's contributions, per entry */
      double dcm[3];
      for (int k = 0; k < 3; ++k) dcm[k] = 0x1p-6 * s->wts[i] * fabs(gC[k]);
      sample_backward_magnitude(lv, 2 * L, mlp, s->idx + 8 * L * i, s->w + 8 * L * i,
                                s->e + 2 * L * i, s->h1 + OR_HIDDEN * nh * i, s->y + OR_DOUT * i,
                                s->h2 + OR_HIDDEN * i, s->sigma[i], s->rgb + 3 * i,
                                s->rgbc + 3 * i, 0x1p-6 * s->dsig_m[i], dcm, 1, bam);
    }
    if (sm < kTie) {
      double dc[3];
      for (int k = 0; k < 3; ++k) dc[k] = s->wts[i] * gC[k];
      sample_tie_deltas(lv, 2 * L, mlp, s->idx + 8 * L * i, s->w + 8 * L * i, s->e + 2 * L * i,
                        s->h1 + OR_HIDDEN * nh * i, s->y + OR_DOUT * i, s->h2 + OR_HIDDEN * i,
                        s->sigma[i], s->rgb + 3 * i, s->rgbc + 3 * i, s->dsig[i], dc, F, kTie, amb);
    }
  }
  return rm;
}

/* Sums per-thread buffers (P floats each) in thread order into out. */
static void reduce_threads(const double* t, int nthreads, int64_t P, double* out) {
  for (int64_t i = 0; i < P; ++i) {
    double acc = 0.0;
    for (int k = 0; k < nthreads; ++k) acc += t[(int64_t)k * P + i];
    out[i] = acc;
  }
}

int or_object_step(const or_config* cfg, const or_levels* lv, int obj, int instance,
                   const float half[3], int nkf, const or_keyframe* kfs, int step, int B,
                   const double* params, const uint8_t* occ, double* grad, double* grad_abs,
                   double* ambiguous, double* bf16_allow, double* min_margin, double* loss,
                   double* loss_allow, or_ray* rays, int nthreads) {
  if (nkf < 1 || B < 1 || cfg->N < 1) return -1;
  const int L = lv->L, N = cfg->N;
  const int64_t P = or_grid_params(lv) + or_mlp_params(2 * L, lv->mlp_layers);
  if (nthreads < 1) nthreads = 1;
  double* ray_loss = (double*)calloc((size_t)B, sizeof(double));
  double* ray_margin = (double*)calloc((size_t)B, sizeof(double));
  double* ray_lallow = (double*)calloc((size_t)B, sizeof(double));
  double* tgrad = NULL;
  double* tabs = NULL;
  double* tamb = NULL;
  if (grad) tgrad = (double*)calloc((size_t)P * nthreads, sizeof(double));
  if (grad && grad_abs) tabs = (double*)calloc((size_t)P * nthreads, sizeof(double));
  double* tbam = NULL;
  if (grad && ambiguous) tamb = (double*)calloc((size_t)P * nthreads, sizeof(double));
  if (grad && bf16_allow) tbam = (double*)calloc((size_t)P * nthreads, sizeof(double));
  if (ambiguous) memset(ambiguous, 0, sizeof(double) * (size_t)P);
  if (bf16_allow) memset(bf16_allow, 0, sizeof(double) * (size_t)P);

#pragma omp parallel num_threads(nthreads)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    or_scratch s;
    scratch_alloc(&s, N, L, lv->mlp_layers);
    double* my_grad = grad ? tgrad + (int64_t)tid * P : NULL;
    double* my_abs = tabs ? tabs + (int64_t)tid * P : NULL;
    double* my_amb = tamb ? tamb + (int64_t)tid * P : NULL;
    double* my_bam = tbam ? tbam + (int64_t)tid * P : NULL;
#pragma omp for schedule(static)
    for (int r = 0; r < B; ++r) {
      or_ray ray;
      or_draw_ray(cfg, obj, step, r, nkf, kfs, instance, &ray);
      const or_keyframe* kf = &kfs[ray.kf];
      or_pixel_ray(kf->M, kf->c, kf->fx, kf->fy, kf->cx, kf->cy, ray.u, ray.v, ray.o, ray.d);
      ray.hit = or_slab(ray.o, ray.d, half, &ray.tn, &ray.tf);
      ray.loss = 0.0;
      ray_lallow[r] = 0.0;
      /* occluder rays carry no loss (Sec. V-B); rays missing the box have no samples */
      if (ray.cls != 0 && ray.hit) {
        double crand[3] = {ray.Crand[0], ray.Crand[1], ray.Crand[2]};
        const int bg = ray.cls == 2;
        ray_forward(lv, N, params, ray.o, ray.d, half, ray.tn, ray.tf, &ray.delta, &s, bg, crand,
                    ray.Chat, &ray.Dhat, &ray.Tend, occ);
        /* Eq. 7-11: squared colour error against the image (object rays) or
         * the random colour (background rays); depth and density terms. */
        double target[3];
        for (int k = 0; k < 3; ++k) target[k] = bg ? crand[k] : (double)ray.C[k];
        double l = 0.0;
        for (int k = 0; k < 3; ++k) l += (ray.Chat[k] - target[k]) * (ray.Chat[k] - target[k]);
        if (!bg && ray.has_depth) l += cfg->lambda_depth * fabs(ray.Dhat - (double)ray.D);
        if (bg) {
          double ssum = 0.0;
          for (int i = 0; i < N; ++i) ssum += s.sigma[i];
          l += cfg->lambda_density * ssum;
        }
        ray.loss = l / (double)B;
        double gC[3], gCm[3], gD = 0.0;
        for (int k = 0; k < 3; ++k) {
          gC[k] = 2.0 * (ray.Chat[k] - target[k]) / (double)B;
          /* the residual's terms: the colour (its samples' and, on a background
           * ray, T_end C_rand) and the target; where they cancel, rounding of
           * the colour moves gC and with it every term of the ray */
          gCm[k] = 2.0 * (fabs(ray.Chat[k]) + fabs(target[k])) / (double)B;
        }
        if (!bg && ray.has_depth) {
          double diff = ray.Dhat - (double)ray.D;
          gD = cfg->lambda_depth * (diff > 0.0 ? 1.0 : (diff < 0.0 ? -1.0 : 0.0)) / (double)B;
        }
        if (my_grad)
          ray_backward(lv, N, params, (double)ray.delta, &s, bg, crand, ray.Tend, gC, gCm, gD,
                       0.0, bg ? cfg->lambda_density / (double)B : 0.0, my_grad, my_abs);
        /* tests only: what the BF16 decisions and the ties can move */
        double dC[3] = {0.0, 0.0, 0.0}, dD = 0.0, dT = 0.0, dS = 0.0;
        if (lv->mlp_bf16 && (loss_allow || my_amb || my_bam))
          bf16_ray_allowance(lv, N, params, &s, (double)ray.delta, bg, crand, ray.Tend, gC, gD,
                             0.0, 1, target, 1.0 / (double)B, my_grad ? my_bam : NULL, dC, &dD,
                             &dT, &dS);
        double la = 0.0;
        for (int k = 0; k < 3; ++k)
          la += 2.0 * fabs(ray.Chat[k] - target[k]) * dC[k] + dC[k] * dC[k];
        if (!bg && ray.has_depth) la += cfg->lambda_depth * dD;
        if (bg) la += cfg->lambda_density * dS;
        ray_lallow[r] = la / (double)B;
        double dtie = INFINITY;
        if (!bg && ray.has_depth)
          dtie = (fabs(ray.Dhat - (double)ray.D) - dD) / fmax(fabs((double)ray.D), 1e-30);
        const double rm = tie_allowance(lv, N, params, &s, gC, dtie, my_grad ? my_amb : NULL,
                                        my_grad ? my_bam : NULL);
        ray_margin[r] = rm;
      } else {
        ray_margin[r] = INFINITY;
      }
      ray_loss[r] = ray.loss;
      if (rays) rays[r] = ray;
    }
    scratch_free(&s);
  }
  double total = 0.0, mm = INFINITY, tla = 0.0;
  for (int r = 0; r < B; ++r) {
    total += ray_loss[r];
    tla += ray_lallow[r];
    mm = fmin(mm, ray_margin[r]);
  }
  *loss = total;
  if (loss_allow) *loss_allow = tla;
  if (min_margin) *min_margin = mm;
  if (grad) reduce_threads(tgrad, nthreads, P, grad);
  if (tabs) reduce_threads(tabs, nthreads, P, grad_abs);
  if (tamb) reduce_threads(tamb, nthreads, P, ambiguous);
  if (tbam) reduce_threads(tbam, nthreads, P, bf16_allow);
  free(tgrad);
  free(tabs);
  free(tamb);
  free(tbam);
  free(ray_loss);
  free(ray_margin);
  free(ray_lallow);
  return 0;
}

/* The field as a differentiable function of the parameters: rays given in the
 * object frame (n x 8 floats: origin, unit direction, t_near, t_far; an empty
 * interval renders nothing), composited on black.  Forward writes rgb (n x 3),
 * depth (n), T_end (n); with grad it also writes the gradient of
 * sum_r (d_rgb_r . C_r + d_depth_r D_r + d_tend_r T_end_r). */
int or_field(const or_config* cfg, const or_levels* lv, const float half[3], const double* params,
             int n, const float* rays, double* rgb, double* depth, double* tend,
             const double* d_rgb, const double* d_depth, const double* d_tend, double* grad,
             double* grad_abs, double* ambiguous, double* bf16_allow, int nthreads) {
  const int L = lv->L, N = cfg->N;
  const int64_t P = or_grid_params(lv) + or_mlp_params(2 * L, lv->mlp_layers);
  if (nthreads < 1) nthreads = 1;
  double* tgrad = grad ? (double*)calloc((size_t)P * nthreads, sizeof(double)) : NULL;
  double* tabs = (grad && grad_abs) ? (double*)calloc((size_t)P * nthreads, sizeof(double)) : NULL;
  double* tamb = (grad && ambiguous) ? (double*)calloc((size_t)P * nthreads, sizeof(double)) : NULL;
  double* tbam = (grad && bf16_allow) ? (double*)calloc((size_t)P * nthreads, sizeof(double)) : NULL;
  if (ambiguous) memset(ambiguous, 0, sizeof(double) * (size_t)P);
  if (bf16_allow) memset(bf16_allow, 0, sizeof(double) * (size_t)P);
#pragma omp parallel num_threads(nthreads)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    or_scratch s;
    scratch_alloc(&s, N, L, lv->mlp_layers);
#pragma omp for schedule(static)
    for (int r = 0; r < n; ++r) {
      const float* q = rays + 8 * (int64_t)r;
      const double zero[3] = {0.0, 0.0, 0.0};
      double C[3] = {0.0, 0.0, 0.0}, D = 0.0, Tend = 1.0;
      float delta = 0.0f;
      const int hit = q[7] > q[6];
      if (hit)
        ray_forward(lv, N, params, q, q + 3, half, q[6], q[7], &delta, &s, 0, zero, C, &D, &Tend,
                    NULL);
      for (int k = 0; k < 3; ++k) rgb[3 * r + k] = C[k];
      depth[r] = D;
      tend[r] = Tend;
      if (grad && hit) {
        const double gC[3] = {d_rgb ? d_rgb[3 * r] : 0.0, d_rgb ? d_rgb[3 * r + 1] : 0.0,
                              d_rgb ? d_rgb[3 * r + 2] : 0.0};
        ray_backward(lv, N, params, (double)delta, &s, 0, zero, Tend, gC, NULL,
                     d_depth ? d_depth[r] : 0.0, d_tend ? d_tend[r] : 0.0, 0.0,
                     tgrad + (int64_t)tid * P, tabs ? tabs + (int64_t)tid * P : NULL);
        double* my_amb = tamb ? tamb + (int64_t)tid * P : NULL;
        double* my_bam = tbam ? tbam + (int64_t)tid * P : NULL;
        if ((my_amb || my_bam) && lv->mlp_bf16) {
          double dC[3], dD, dT, dS;
          bf16_ray_allowance(lv, N, params, &s, (double)delta, 0, zero, Tend, gC,
                             d_depth ? d_depth[r] : 0.0, d_tend ? d_tend[r] : 0.0, 0, zero, 0.0,
                             my_bam, dC, &dD, &dT, &dS);
        }
        if (my_amb) tie_allowance(lv, N, params, &s, gC, INFINITY, my_amb, my_bam);
      }
    }
    scratch_free(&s);
  }
  if (grad) reduce_threads(tgrad, nthreads, P, grad);
  if (tabs) reduce_threads(tabs, nthreads, P, grad_abs);
  if (tamb) reduce_threads(tamb, nthreads, P, ambiguous);
  if (tbam) reduce_threads(tbam, nthreads, P, bf16_allow);
  free(tgrad);
  free(tabs);
  free(tamb);
  free(tbam);
  return 0;
}

/* Dense Adam (the paper's "backward and optimization" phase; optimiser not
 * named).  k is the step number after increment (1 on the first step). */
void or_adam(int64_t P, double* p, double* g, double* m, double* v, int k, double lr, double b1,
             double b2, double eps) {
  double bc1 = 1.0 - pow(b1, (double)k);
  double bc2 = 1.0 - pow(b2, (double)k);
  for (int64_t i = 0; i < P; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / bc1) / (sqrt(v[i] / bc2) + eps);
    g[i] = 0.0;
  }
}

/* Render every pixel of a camera through the object's box (evaluation and
 * meshing); composited on black, opacity = 1 - T_end.  Misses give 0.
 * rgb_allow (tests only, may be NULL; BF16 mode): per pixel and channel the
 * bound of the change of the colour under the other choice of the
 * ambiguous BF16 roundings (bf16_ray_allowance); 0 in FP32 mode. */
int or_render(const or_config* cfg, const or_levels* lv, const float half[3],
              const or_keyframe* cam, const double* params, const uint8_t* occ, double* rgb,
              double* depth, double* opacity, double* rgb_allow, int nthreads) {
  const int L = lv->L, N = cfg->N;
  const int64_t npix = (int64_t)cam->W * cam->H;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
  {
    or_scratch s;
    scratch_alloc(&s, N, L, lv->mlp_layers);
#pragma omp for schedule(static)
    for (int64_t px = 0; px < npix; ++px) {
      int u = (int)(px % cam->W), v = (int)(px / cam->W);
      float o[3], d[3], tn, tf, dl;
      or_pixel_ray(cam->M, cam->c, cam->fx, cam->fy, cam->cx, cam->cy, u, v, o, d);
      double C[3] = {0.0, 0.0, 0.0}, D = 0.0, Tend = 1.0, dC[3] = {0.0, 0.0, 0.0};
      if (or_slab(o, d, half, &tn, &tf)) {
        const double zero[3] = {0.0, 0.0, 0.0};
        ray_forward(lv, N, params, o, d, half, tn, tf, &dl, &s, 0, zero, C, &D, &Tend, occ);
        if (rgb_allow && lv->mlp_bf16) {
          double dD, dT, dS;
          bf16_ray_allowance(lv, N, params, &s, (double)dl, 0, zero, Tend, zero, 0.0, 0.0, 0,
                             zero, 0.0, NULL, dC, &dD, &dT, &dS);
        }
      }
      for (int k = 0; k < 3; ++k) rgb[3 * px + k] = C[k];
      if (rgb_allow)
        for (int k = 0; k < 3; ++k) rgb_allow[3 * px + k] = dC[k];
      if (depth) depth[px] = D;
      if (opacity) opacity[px] = 1.0 - Tend;
    }
    scratch_free(&s);
  }
  return 0;
}

/* Density at object-frame points (used for meshing by marching cubes). */
void or_query_density(const or_levels* lv, const float half[3], const double* params, int64_t n,
                      const float* xyz, double* sigma) {
  const int din = 2 * lv->L;
  const double* mlp = params + or_grid_params(lv);
  uint32_t idx[8 * OR_MAX_LEVELS];
  double w[8 * OR_MAX_LEVELS], e[2 * OR_MAX_LEVELS], h1[OR_HIDDEN * OR_MAX_MLP_LAYERS], y[OR_DOUT],
      h2[OR_HIDDEN], rgb[3];
  for (int64_t i = 0; i < n; ++i) {
    float p[3];
    for (int k = 0; k < 3; ++k) {
      float q = (xyz[3 * i + k] + half[k]) / (half[k] + half[k]);
      p[k] = fminf(fmaxf(q, 0.0f), 1.0f);
    }
    or_encode(lv, p, params, idx, w, e);
    /* the density query runs the FP32 MLP in either mode */
    or_mlp_forward(din, lv->mlp_layers, 0, mlp, e, h1, y, h2, sigma + i, rgb, NULL);
  }
}

/* ------------------------------------------------------------------------
 * Marching cubes (Lorensen & Cline 1987), the mesh extraction of Sec. III
 * (64^3 per object in Sec. VI; meshes placed in the world by the object pose).
 *
 * Cell corners are numbered by their offsets, corner c = (c&1, c>>1&1, c>>2&1).
 * Edges: 0..3 along x from corners 0,2,4,6; 4..7 along y from corners
 * 0,1,4,5; 8..11 along z from corners 0,1,2,3.  A corner is inside when its
 * value is > iso.  The triangles of a case are derived, not tabulated from
 * elsewhere: the crossing points (one per edge whose ends differ) are joined
 * into closed loops face by face -- on a face with two crossings the two are
 * joined; on a face with four (the ambiguous pattern) each inside corner of
 * the face is cut off by joining its two edges -- and every loop becomes a
 * triangle fan.  Canonical form of a loop: oriented so that its normal
 * (Newell's method over the edge midpoints) points from the inside end of
 * its first edge to the outside end, then rotated to start at its smallest
 * edge number; loops are emitted by increasing smallest edge number, each as
 * a fan from its first vertex (in that order) whose fan has no triangle
 * lying in a cube face: (v_a, v_a+i, v_a+i+1), i = 1 .. len-2.
 * ---------------------------------------------------------------------- */

static const int or_mc_edge_end[12][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3},
                                          {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
/* the 6 faces as corner cycles */
static const int or_mc_face[6][4] = {{0, 2, 6, 4}, {1, 3, 7, 5}, {0, 1, 5, 4},
                                     {2, 3, 7, 6}, {0, 1, 3, 2}, {4, 5, 7, 6}};

static int or_mc_edge_of(int a, int b) {
  for (int e = 0; e < 12; ++e)
    if ((or_mc_edge_end[e][0] == a && or_mc_edge_end[e][1] == b) ||
        (or_mc_edge_end[e][0] == b && or_mc_edge_end[e][1] == a))
      return e;
  return -1;
}

static int or_mc_edge_on_face(int e, int f) {
  int hits = 0;
  for (int i = 0; i < 4; ++i)
    hits += (or_mc_face[f][i] == or_mc_edge_end[e][0]) + (or_mc_face[f][i] == or_mc_edge_end[e][1]);
  return hits == 2;
}

static int8_t or_mc_tris[256][16]; /* edge triples, -1 terminated */
static int or_mc_ntri[256];
static int or_mc_built = 0;

static void or_mc_build(void) {
  for (int m = 0; m < 256; ++m) {
    int nb[12][2], nn[12];
    for (int e = 0; e < 12; ++e) nn[e] = 0;
    for (int f = 0; f < 6; ++f) {
      const int* cyc = or_mc_face[f];
      int ce[4], in[4], k = 0;
      for (int i = 0; i < 4; ++i) in[i] = (m >> cyc[i]) & 1;
      int side[4];
      for (int i = 0; i < 4; ++i) {
        side[i] = or_mc_edge_of(cyc[i], cyc[(i + 1) & 3]); /* edge between cyc[i], cyc[i+1] */
        if (in[i] != in[(i + 1) & 3]) ce[k++] = side[i];
      }
      int pa[2][2], np = 0;
      if (k == 2) {
        pa[0][0] = ce[0];
        pa[0][1] = ce[1];
        np = 1;
      } else if (k == 4) { /* inside corners cut off by their two edges */
        if (in[0]) {
          pa[0][0] = side[3]; pa[0][1] = side[0];
          pa[1][0] = side[1]; pa[1][1] = side[2];
        } else {
          pa[0][0] = side[0]; pa[0][1] = side[1];
          pa[1][0] = side[2]; pa[1][1] = side[3];
        }
        np = 2;
      }
      for (int j = 0; j < np; ++j) {
        const int a = pa[j][0], b = pa[j][1];
        nb[a][nn[a]++] = b;
        nb[b][nn[b]++] = a;
      }
    }
    int used[12] = {0}, nt = 0;
    int loops[12][12], llen[12], nl = 0;
    for (int e0 = 0; e0 < 12; ++e0) {
      if (nn[e0] == 0 || used[e0]) continue;
      int len = 0, prev = -1, cur = e0;
      /* walk from e0 towards its smaller-numbered neighbour first */
      int first = nb[e0][0] < nb[e0][1] ? nb[e0][0] : nb[e0][1];
      loops[nl][len++] = e0;
      used[e0] = 1;
      prev = e0;
      cur = first;
      while (cur != e0) {
        loops[nl][len++] = cur;
        used[cur] = 1;
        const int nx = nb[cur][0] == prev ? nb[cur][1] : nb[cur][0];
        prev = cur;
        cur = nx;
      }
      llen[nl++] = len;
    }
    for (int L = 0; L < nl; ++L) {
      int* lp = loops[L];
      const int len = llen[L];
      /* Newell normal over the edge midpoints */
      double nrm[3] = {0, 0, 0};
      for (int i = 0; i < len; ++i) {
        double p[3], q[3];
        for (int k = 0; k < 3; ++k) {
          const int a0 = or_mc_edge_end[lp[i]][0], a1 = or_mc_edge_end[lp[i]][1];
          const int b0 = or_mc_edge_end[lp[(i + 1) % len]][0],
                    b1 = or_mc_edge_end[lp[(i + 1) % len]][1];
          p[k] = 0.5 * (((a0 >> k) & 1) + ((a1 >> k) & 1));
          q[k] = 0.5 * (((b0 >> k) & 1) + ((b1 >> k) & 1));
        }
        nrm[0] += (p[1] - q[1]) * (p[2] + q[2]);
        nrm[1] += (p[2] - q[2]) * (p[0] + q[0]);
        nrm[2] += (p[0] - q[0]) * (p[1] + q[1]);
      }
      const int c0 = or_mc_edge_end[lp[0]][0], c1 = or_mc_edge_end[lp[0]][1];
      const int cin = ((m >> c0) & 1) ? c0 : c1, cout = cin == c0 ? c1 : c0;
      double dot = 0;
      for (int k = 0; k < 3; ++k) dot += nrm[k] * (double)(((cout >> k) & 1) - ((cin >> k) & 1));
      if (dot < 0) { /* reverse */
        for (int i = 0; i < len / 2; ++i) {
          const int t = lp[i];
          lp[i] = lp[len - 1 - i];
          lp[len - 1 - i] = t;
        }
      }
      int s = 0;
      for (int i = 1; i < len; ++i)
        if (lp[i] < lp[s]) s = i;
      int rot[12];
      for (int i = 0; i < len; ++i) rot[i] = lp[(s + i) % len];
      for (int i = 0; i < len; ++i) lp[i] = rot[i];
    }
    /* loops by increasing first (smallest) edge */
    for (int a = 0; a < nl; ++a)
      for (int b = a + 1; b < nl; ++b)
        if (loops[b][0] < loops[a][0]) {
          int tmp[12], tl = llen[a];
          for (int i = 0; i < 12; ++i) tmp[i] = loops[a][i];
          for (int i = 0; i < 12; ++i) loops[a][i] = loops[b][i];
          llen[a] = llen[b];
          for (int i = 0; i < 12; ++i) loops[b][i] = tmp[i];
          llen[b] = tl;
        }
    for (int L = 0; L < nl; ++L) {
      /* fan apex: the first loop vertex from which no fan triangle lies in a
       * cube face (a face holding two segments of the loop would otherwise
       * get a flat triangle, duplicated by the neighbouring cell) */
      const int len = llen[L];
      int apex = 0;
      for (int s0 = 0; s0 < len; ++s0) {
        int flat = 0;
        for (int i = 1; i + 1 < len && !flat; ++i)
          for (int f = 0; f < 6; ++f)
            if (or_mc_edge_on_face(loops[L][s0], f) &&
                or_mc_edge_on_face(loops[L][(s0 + i) % len], f) &&
                or_mc_edge_on_face(loops[L][(s0 + i + 1) % len], f))
              flat = 1;
        if (!flat) {
          apex = s0;
          break;
        }
      }
      for (int i = 1; i + 1 < len; ++i) {
        or_mc_tris[m][3 * nt] = (int8_t)loops[L][apex];
        or_mc_tris[m][3 * nt + 1] = (int8_t)loops[L][(apex + i) % len];
        or_mc_tris[m][3 * nt + 2] = (int8_t)loops[L][(apex + i + 1) % len];
        ++nt;
      }
    }
    for (int i = 3 * nt; i < 16; ++i) or_mc_tris[m][i] = -1;
    or_mc_ntri[m] = nt;
  }
  or_mc_built = 1;
}

int or_mc_case(int m, int8_t tris[16]) {
  if (!or_mc_built) or_mc_build();
  for (int i = 0; i < 16; ++i) tris[i] = or_mc_tris[m & 255][i];
  return or_mc_ntri[m & 255];
}

/* grid: (res+1)^3 values, x fastest, corner (i,j,k) at lo + (hi - lo) * (i,j,k)/res
 * (FP32, that expression order).  Writes up to max_tris triangles (9 floats:
 * three vertices) in cell order (x fastest), returns the total count.  Vertex
 * on an edge from corner a to corner b: t = (iso - v_a) / (v_b - v_a),
 * x = x_a + t * (x_b - x_a), FP32, no contraction. */
int64_t or_marching_cubes(const float* grid, int res, float iso, const float lo[3],
                          const float hi[3], float* out, int64_t max_tris) {
  if (!or_mc_built) or_mc_build();
  const int64_t n1 = res + 1;
  int64_t total = 0;
  for (int k = 0; k < res; ++k)
    for (int j = 0; j < res; ++j)
      for (int i = 0; i < res; ++i) {
        float v[8], x[8][3];
        int m = 0;
        for (int c = 0; c < 8; ++c) {
          const int ci = i + (c & 1), cj = j + ((c >> 1) & 1), ck = k + ((c >> 2) & 1);
          v[c] = grid[(int64_t)ci + n1 * ((int64_t)cj + n1 * ck)];
          const int g[3] = {ci, cj, ck};
          for (int a = 0; a < 3; ++a) x[c][a] = lo[a] + (hi[a] - lo[a]) * ((float)g[a] / (float)res);
          if (v[c] > iso) m |= 1 << c;
        }
        for (int t = 0; t < or_mc_ntri[m]; ++t, ++total) {
          if (!out || total >= max_tris) continue;
          for (int q = 0; q < 3; ++q) {
            const int e = or_mc_tris[m][3 * t + q];
            const int a = or_mc_edge_end[e][0], b = or_mc_edge_end[e][1];
            const float s = (iso - v[a]) / (v[b] - v[a]);
            for (int d = 0; d < 3; ++d) out[9 * total + 3 * q + d] = x[a][d] + s * (x[b][d] - x[a][d]);
          }
        }
      }
  return total;
}

/* ------------------------------------------------------------------------
 * Object box from its sparse point cloud (Sec. IV-B, pose and size
 * estimation): translation = midpoint of the per-axis extremes of the world
 * points (Eq. 1); yaw = direction of the dominant principal axis of the
 * points projected on the horizontal plane (PCA), folded into [-pi/2, pi/2)
 * (a cuboid's axis has no sign); size = half the per-axis extent of the
 * points in the object frame rotated by that yaw (Eq. 4).  Roll and pitch
 * are zero (objects on a support).  FP64 throughout.  The line-feature
 * refinement of the yaw (Eq. 2-3) needs image line segments and is not
 * computed here.
 * ---------------------------------------------------------------------- */
int or_box_from_points(const double* xyz, int64_t n, double t[3], double* yaw, double half[3]) {
  if (n < 1) return -1;
  double mn[3], mx[3];
  for (int k = 0; k < 3; ++k) mn[k] = mx[k] = xyz[k];
  for (int64_t i = 1; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      const double v = xyz[3 * i + k];
      if (v < mn[k]) mn[k] = v;
      if (v > mx[k]) mx[k] = v;
    }
  for (int k = 0; k < 3; ++k) t[k] = 0.5 * (mx[k] + mn[k]); /* Eq. 1 */
  /* PCA of the horizontal projection: 2x2 covariance about the mean */
  double mxy[2] = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    mxy[0] += xyz[3 * i];
    mxy[1] += xyz[3 * i + 1];
  }
  mxy[0] /= (double)n;
  mxy[1] /= (double)n;
  double sxx = 0, syy = 0, sxy = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double dx = xyz[3 * i] - mxy[0], dy = xyz[3 * i + 1] - mxy[1];
    sxx += dx * dx;
    syy += dy * dy;
    sxy += dx * dy;
  }
  /* eigenvector of the larger eigenvalue of [[sxx, sxy], [sxy, syy]] is at
   * angle 0.5 * atan2(2 sxy, sxx - syy) */
  double th = 0.5 * atan2(2.0 * sxy, sxx - syy);
  const double pi = 3.14159265358979323846;
  if (th >= 0.5 * pi) th -= pi;
  if (th < -0.5 * pi) th += pi;
  *yaw = th;
  const double c = cos(th), s = sin(th);
  double lo[3], hi[3];
  for (int64_t i = 0; i < n; ++i) {
    const double dx = xyz[3 * i] - t[0], dy = xyz[3 * i + 1] - t[1], dz = xyz[3 * i + 2] - t[2];
    const double o[3] = {c * dx + s * dy, -s * dx + c * dy, dz}; /* R(yaw)^T (x - t) */
    for (int k = 0; k < 3; ++k) {
      if (i == 0 || o[k] < lo[k]) lo[k] = o[k];
      if (i == 0 || o[k] > hi[k]) hi[k] = o[k];
    }
  }
  for (int k = 0; k < 3; ++k) half[k] = 0.5 * (hi[k] - lo[k]); /* Eq. 4 */
  return 0;
}
