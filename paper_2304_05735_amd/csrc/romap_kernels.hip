// romap_kernels.hip -- gfx950 kernels of one training step of RO-MAP's
// per-object radiance fields (arXiv 2304.05735, Sec. V).
//
// One step over every object of a launch:
//   k_raygen       draw rays in each object's detection boxes, classify them by
//                  the instance mask, back-project into the object frame, clip
//                  to the 3D box (Sec. V-B)                        [FP32, exact]
//   k_encode_fwd   multiresolution hash-grid gather, one (object, level) table
//                  at a time
//   k_pack         MLP weights -> MFMA operand images (FP32 and BF16); advances
//                  the Adam step
//   k_field        fused per-ray MLP (MFMA) + volume rendering (Eq. 6) + loss
//                  (Eq. 7-11) + adjoint, activations recomputed in the backward
//                  half, wavefront prefix scans for transmittance
//   k_reduce       per-object MLP gradient and loss from the work-item records;
//                  Adam on the MLP weights
//   k_bin_scatter  encoding adjoint -> (entry, value) records sorted into bins
//                  of table regions
//   k_bin_acc      region sums in LDS; Adam on the region's table entries
//   k_bin_finish   Adam on regions summed by several workgroups
//
// Adam is dense: every parameter of every object of the step is updated each
// step, each where its gradient is complete, so the gradient itself is never
// written in a training step.
//
// Precision: the ray / sample-position / cell / hash path is IEEE FP32 with no
// contraction (this file is built with -ffp-contract=off; FMAs are written
// out where wanted), so positions and indices are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <math.h>
#include <stdint.h>

#include "romap_device.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// small helpers

// Philox4x32-10 (Salmon et al., SC'11): the counter-based generator behind
// every random draw, so a draw depends only on (seed, object, step, ray).
__device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx2_t __attribute__((ext_vector_type(2)));

// FP32 -> BF16 with round to nearest, ties to even (gfx950 v_cvt_pk_bf16_f32)
__device__ inline uint32_t pack_bf16x2(float x, float y) {
  const floatx2_t v = {x, y};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// FP32 -> BF16, round to nearest even (integer form, for the weight images)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Orders this wave's LDS traffic: every lane's earlier LDS accesses are
// complete before any lane's later ones (cross-lane exchange inside a wave).
// Orders a wave's LDS writes before its later LDS reads of other lanes' data
// (and reads before later writes): the LDS executes one wave's operations in
// issue order, so only the compiler must keep them in program order; the
// hardware waits where a read's result is used.
__device__ inline void wave_lds_sync() { asm volatile("" ::: "memory"); }

// Wave-wide scans in registers with DPP (no LDS round trips): row shifts
// build the scan inside each 16-lane row, row broadcasts carry the row
// totals across.  Lanes a shift reads from outside the row (or the wave)
// read 0.
template <int CTRL, int ROWM = 0xf, int BANKM = 0xf, bool BC = true>
__device__ inline float dppf(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWM, BANKM, BC));
}

__device__ inline float readlane_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// inclusive prefix sum over the 64 lanes
__device__ inline float wave_incl_prefix(float x) {
  x += dppf<0x111>(x);                   // row_shr:1
  x += dppf<0x112>(x);                   // row_shr:2
  x += dppf<0x114>(x);                   // row_shr:4
  x += dppf<0x118>(x);                   // row_shr:8
  x += dppf<0x142, 0xa, 0xf, false>(x);  // row_bcast:15 into rows 1 and 3
  x += dppf<0x143, 0xc, 0xf, false>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ inline float wave_sum(float x) { return readlane_f(wave_incl_prefix(x), 63); }

// exclusive suffix sum over the 64 lanes (sum over lanes > lane)
__device__ inline float wave_excl_suffix(float x, int lane) {
  x += dppf<0x101>(x);  // row_shl:1
  x += dppf<0x102>(x);  // row_shl:2
  x += dppf<0x104>(x);  // row_shl:4
  x += dppf<0x108>(x);  // row_shl:8: inclusive suffix inside the row
  const float t1 = readlane_f(x, 16), t2 = readlane_f(x, 32), t3 = readlane_f(x, 48);
  const int row = lane >> 4;
  x += row == 0 ? (t1 + t2) + t3 : (row == 1 ? t2 + t3 : (row == 2 ? t3 : 0.0f));
  return dppf<0x130>(x);  // wave_shl:1: the next lane's inclusive suffix
}

// integer inclusive prefix sum over the 64 lanes (same steps)
template <int CTRL, int ROWM = 0xf, int BANKM = 0xf, bool BC = true>
__device__ inline int dppi(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWM, BANKM, BC);
}

__device__ inline int wave_incl_prefix_i(int x) {
  x += dppi<0x111>(x);
  x += dppi<0x112>(x);
  x += dppi<0x114>(x);
  x += dppi<0x118>(x);
  x += dppi<0x142, 0xa, 0xf, false>(x);
  x += dppi<0x143, 0xc, 0xf, false>(x);
  return x;
}

// exclusive prefix without the subtraction: shift the inclusive scan by one lane
__device__ inline float wave_excl_prefix(float x, int lane) {
  return dppf<0x138>(wave_incl_prefix(x));  // wave_shr:1
}

// Position of sample i of a ray in the unit cube of the object's box:
// d_i = t_n + (i + 1/2) delta, x = o + d_i d, p = (x + a) / 2a, clamped.
__device__ inline void sample_pos(const RayRec& R, int i, const float* half, float p[3]) {
  const float di = R.tn + ((float)i + 0.5f) * R.delta;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float x = R.o[k] + di * R.d[k];
    const float q = (x + half[k]) / (half[k] + half[k]);
    p[k] = fminf(fmaxf(q, 0.0f), 1.0f);
  }
}

// Occupancy skip: 64^3 bits over the unit cube, bit x + 64 y + 4096 z of cell
// floor(64 p) (clamped).  A sample in a clear cell has density 0.
__device__ inline bool occupied(const uint32_t* occ, const float p[3]) {
  if (!occ) return true;
  int c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int ci = (int)floorf(p[k] * 64.0f);
    c[k] = ci < 0 ? 0 : (ci > 63 ? 63 : ci);
  }
  const int bit = c[0] + 64 * c[1] + 4096 * c[2];
  return (occ[bit >> 5] >> (bit & 31)) & 1u;
}

struct Cell {
  uint32_t c[3];
  float f[3];
};

__device__ inline void make_cell(const float p[3], uint32_t N, Cell& cl) {
  const float Nf = (float)N;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float g = p[k] * Nf;
    int ci = (int)floorf(g);
    ci = ci < 0 ? 0 : ci;
    ci = ci > (int)N - 1 ? (int)N - 1 : ci;
    cl.c[k] = (uint32_t)ci;
    cl.f[k] = g - (float)ci;
  }
}

// Index of corner b (bit0 x, bit1 y, bit2 z) of a cell within its level:
// dense 1:1 when the level fits its table, else the spatial hash of the
// multiresolution hash encoding (primes 1, 2654435761, 805459861) mod T.
__device__ inline uint32_t corner_index(const Cell& cl, int b, uint32_t N, uint32_t T,
                                        bool hashed) {
  const uint32_t vx = cl.c[0] + (uint32_t)(b & 1);
  const uint32_t vy = cl.c[1] + (uint32_t)((b >> 1) & 1);
  const uint32_t vz = cl.c[2] + (uint32_t)((b >> 2) & 1);
  if (hashed) return (vx ^ (vy * 2654435761u) ^ (vz * 805459861u)) & (T - 1u);
  const uint32_t n1 = N + 1u;
  return vx + vy * n1 + vz * n1 * n1;
}

__device__ inline float corner_weight(const Cell& cl, int b) {
  const float wx = (b & 1) ? cl.f[0] : 1.0f - cl.f[0];
  const float wy = (b & 2) ? cl.f[1] : 1.0f - cl.f[1];
  const float wz = (b & 4) ? cl.f[2] : 1.0f - cl.f[2];
  return (wx * wy) * wz;
}

// All 8 corner indices of a cell, with the products shared between corners:
// (c + 1) * P = c * P + P mod 2^32 for the hash, and the dense index of
// corner b is the cell's index plus b's offsets.  Same values as corner_index
// for slot b ^ flip: flip = 0 gives the corners in order b, flip = the
// cell's coordinate parities gives parity slots (slot q is the corner whose
// vertex has parities q, the same slot in every cell sharing that vertex).
__device__ inline void cell_corners(const Cell& cl, uint32_t N, uint32_t T, bool hashed,
                                    uint32_t idx[8], uint32_t flip = 0u) {
  // per axis, the two vertex offsets in slot order
  const uint32_t fx = flip & 1u, fy = (flip >> 1) & 1u, fz = (flip >> 2) & 1u;
  if (hashed) {
    const uint32_t xa = cl.c[0], ya = cl.c[1] * 2654435761u, za = cl.c[2] * 805459861u;
    const uint32_t xb = xa + 1u, yb = ya + 2654435761u, zb = za + 805459861u;
    const uint32_t x0 = fx ? xb : xa, x1 = fx ? xa : xb;
    const uint32_t y0 = fy ? yb : ya, y1 = fy ? ya : yb;
    const uint32_t z0 = fz ? zb : za, z1 = fz ? za : zb;
    const uint32_t m = T - 1u;
    idx[0] = (x0 ^ y0 ^ z0) & m;
    idx[1] = (x1 ^ y0 ^ z0) & m;
    idx[2] = (x0 ^ y1 ^ z0) & m;
    idx[3] = (x1 ^ y1 ^ z0) & m;
    idx[4] = (x0 ^ y0 ^ z1) & m;
    idx[5] = (x1 ^ y0 ^ z1) & m;
    idx[6] = (x0 ^ y1 ^ z1) & m;
    idx[7] = (x1 ^ y1 ^ z1) & m;
  } else {
    const uint32_t n1 = N + 1u, n2 = n1 * n1;
    const uint32_t b0 = cl.c[0] + cl.c[1] * n1 + cl.c[2] * n2;
    const uint32_t ox[2] = {fx, 1u - fx}, oy[2] = {fy * n1, (1u - fy) * n1},
                   oz[2] = {fz * n2, (1u - fz) * n2};
#pragma unroll
    for (int b = 0; b < 8; ++b) idx[b] = b0 + ox[b & 1] + oy[(b >> 1) & 1] + oz[b >> 2];
  }
}

// All 8 trilinear weights, (wx * wy) * wz as corner_weight, sharing wx * wy,
// in the slots of cell_corners with the same flip.
__device__ inline void cell_weights(const Cell& cl, float w[8], uint32_t flip = 0u) {
  const float gx = 1.0f - cl.f[0], gy = 1.0f - cl.f[1], gz = 1.0f - cl.f[2];
  const float wx[2] = {(flip & 1u) ? cl.f[0] : gx, (flip & 1u) ? gx : cl.f[0]};
  const float wy[2] = {(flip & 2u) ? cl.f[1] : gy, (flip & 2u) ? gy : cl.f[1]};
  const float wz[2] = {(flip & 4u) ? cl.f[2] : gz, (flip & 4u) ? gz : cl.f[2]};
  float wxy[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wxy[q] = wx[q & 1] * wy[q >> 1];
#pragma unroll
  for (int b = 0; b < 8; ++b) w[b] = wxy[b & 3] * wz[b >> 2];
}

// the cell's coordinate parities (bit k: c_k & 1)
__device__ inline uint32_t cell_parity(const Cell& cl) {
  return (cl.c[0] & 1u) | ((cl.c[1] & 1u) << 1) | ((cl.c[2] & 1u) << 2);
}

__device__ inline int find_sobj(const StepObj* so, int n, int r) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (so[mid].ray_begin <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Back-projection of pixel (u, v) and clipping to the box [-a, a]:
// pinhole camera, pixel centres at +0.5, unit direction, slab test.
__device__ inline void pixel_ray(const float* M, const float* c, float fx, float fy, float cx,
                                 float cy, int u, int v, const float* half, RayRec& R, int NS) {
  const float x = (((float)u + 0.5f) - cx) / fx;
  const float y = (((float)v + 0.5f) - cy) / fy;
  float dd[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) dd[k] = (M[3 * k + 0] * x + M[3 * k + 1] * y) + M[3 * k + 2];
  const float n = sqrtf((dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]);
  float tmin = -INFINITY, tmax = INFINITY;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R.d[k] = dd[k] / n;
    R.o[k] = c[k];
    const float inv = 1.0f / R.d[k];
    const float t0 = (-half[k] - R.o[k]) * inv;
    const float t1 = (half[k] - R.o[k]) * inv;
    tmin = fmaxf(tmin, fminf(t0, t1));
    tmax = fminf(tmax, fmaxf(t0, t1));
  }
  const float tn = fmaxf(tmin, 0.0f);
  const bool hit = tmax > tn;
  R.tn = tn;
  R.delta = hit ? (tmax - tn) / (float)NS : 0.0f;
  R.flags = hit ? RM_F_HIT : 0u;
}

// ---------------------------------------------------------------------------
// K1: ray draw, classification, back-projection, box clipping (Sec. V-B)
template <int NS>
__global__ __launch_bounds__(256) void k_raygen(StepArgs a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n_rays) return;
  const int si = find_sobj(a.sobj, a.n_sobj, r);
  const StepObj so = a.sobj[si];
  const ObjStatic& ob = a.objs[so.obj];
  const int local = r - so.ray_begin;
  const uint32_t step = (uint32_t)a.state[so.obj].step;
  uint32_t x[4];
  philox4x32_10(step, (uint32_t)local, 0u, 0u, a.seed_lo ^ (uint32_t)ob.id, a.seed_hi, x);
  const int64_t q = (int64_t)(((uint64_t)x[0] * (uint64_t)ob.n_cand) >> 32);
  int lo = 0, hi = ob.n_kf - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ob.kfs[mid].cand_begin <= q) lo = mid; else hi = mid - 1;
  }
  const KfRef& kr = ob.kfs[lo];
  const int64_t lq = q - kr.cand_begin;
  const int u = kr.x0 + (int)(lq % kr.w);
  const int v = kr.y0 + (int)(lq / kr.w);
  const KfDev kf = a.kfs[kr.kf];
  float crand[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) crand[j] = (float)(x[j + 1] >> 8) * (1.0f / 16777216.0f);
  const int64_t pix = (int64_t)v * kf.W + u;
  const int m = kf.mask[pix];
  const uint32_t cls = (m == ob.instance) ? RM_CLS_OBJECT : (m == 0 ? RM_CLS_BACKGROUND : RM_CLS_OCCLUDER);
  RayRec R;
  pixel_ray(kr.M, kr.c, kf.fx, kf.fy, kf.cx, kf.cy, u, v, ob.half, R, NS);
  R.flags |= cls;
  R.D = 0.0f;
  if (cls == RM_CLS_BACKGROUND) {
#pragma unroll
    for (int j = 0; j < 3; ++j) R.tgt[j] = crand[j];
  } else {
#pragma unroll
    for (int j = 0; j < 3; ++j) R.tgt[j] = (float)kf.rgb[3 * pix + j] / 255.0f;
  }
  if (cls == RM_CLS_OBJECT && kf.depth) {
    const float z = kf.depth[pix];
    if (z > 0.0f && isfinite(z)) {
      // camera z -> distance along the ray, the quantity of Eq. 8
      const float xn = (((float)u + 0.5f) - kf.cx) / kf.fx;
      const float yn = (((float)v + 0.5f) - kf.cy) / kf.fy;
      R.D = z * sqrtf((xn * xn + yn * yn) + 1.0f);
      R.flags |= RM_F_DEPTH;
    }
  }
  R.obj = so.obj;
  R.pad0 = 0;
  R.pad1 = 0;
  a.rays[r] = R;
  if (a.dbg_kfuv) {
    a.dbg_kfuv[3 * r + 0] = lo;
    a.dbg_kfuv[3 * r + 1] = u;
    a.dbg_kfuv[3 * r + 2] = v;
  }
}

// rays of every pixel of a camera, for rendering (class "object", no target)
struct CamArgs {
  float M[9], c[3];
  float fx, fy, cx, cy;
  int W, pix0;
};

template <int NS>
__global__ __launch_bounds__(256) void k_camera_rays(StepArgs a, CamArgs ca) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n_rays) return;
  const int p = ca.pix0 + r;
  const int obj = a.sobj[0].obj;
  RayRec R;
  pixel_ray(ca.M, ca.c, ca.fx, ca.fy, ca.cx, ca.cy, p % ca.W, p / ca.W, a.objs[obj].half, R, NS);
  R.flags |= RM_CLS_OBJECT;
  R.tgt[0] = R.tgt[1] = R.tgt[2] = 0.0f;
  R.D = 0.0f;
  R.obj = obj;
  R.pad0 = R.pad1 = 0;
  a.rays[r] = R;
}

// caller-given rays (o, d, t_near, t_far) in the object frame
template <int NS>
__global__ __launch_bounds__(256) void k_user_rays(StepArgs a, const float* rays) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n_rays) return;
  const float* q = rays + 8 * (int64_t)r;
  RayRec R;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R.o[k] = q[k];
    R.d[k] = q[3 + k];
  }
  const float tn = q[6], tf = q[7];
  const bool hit = tf > tn;
  R.tn = tn;
  R.delta = hit ? (tf - tn) / (float)NS : 0.0f;
  R.flags = (hit ? RM_F_HIT : 0u) | RM_CLS_OBJECT;
  R.tgt[0] = R.tgt[1] = R.tgt[2] = 0.0f;
  R.D = 0.0f;
  R.obj = a.sobj[0].obj;
  R.pad0 = R.pad1 = 0;
  a.rays[r] = R;
}

__device__ inline bool ray_active(uint32_t flags) {
  return (flags & RM_F_HIT) && (flags & RM_F_CLS) != RM_CLS_OCCLUDER;
}

// ---------------------------------------------------------------------------
// K2: encoding forward.  RM_ENC_SPLIT workgroups per block of RM_SCAT_WG
// samples of one (object, level) pair, blocks ordered object by object and
// level by level within an object, so the chip sweeps one table at a time;
// the object and level are uniform in a workgroup.  blockDim threads cover
// the workgroup's samples.
template <int NS>
__global__ __launch_bounds__(512) void k_encode_fwd(StepArgs a) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = gtid; j < a.n_regions; j += (int64_t)gridDim.x * blockDim.x)
    a.bin_count[j] = 0;  // fresh fill counters for the binned scatter of this pass
  // Workgroup i runs on XCD i mod 8; numbered so that each XCD takes a
  // contiguous range of (object, level) blocks, a level's table is gathered
  // by one XCD at a time and stays in its L2: the L2 hit rate goes from 0.67
  // to 0.93 and the lines fetched beyond the L2 from 2.8 to 0.5 GB per step
  // on the 24-object workload.  The kernel alone is no faster (it is bound by
  // the L2's request rate, the same either way, and the XCDs' ranges differ
  // in cost: 492 -> 522 us), but the bandwidth it no longer takes goes to
  // the other object group's kernels: 1.812 -> 1.800 ms per step.
  const int nwg = a.n_bblocks * RM_ENC_SPLIT;
  const int per_xcd = (nwg + 7) >> 3;
  const int jw = (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3);
  if (jw >= nwg) return;
  const BinBlock bb = a.bblocks[jw / RM_ENC_SPLIT];
  constexpr int SPAN = RM_SCAT_WG / RM_ENC_SPLIT;  // samples of this workgroup
  const int k0 = (jw % RM_ENC_SPLIT) * SPAN;
  const BinPair bp = a.bpairs[bb.pair];
  const ObjStatic& ob = a.objs[a.sobj[bp.so].obj];
  const int l = bp.l;
  const uint32_t N = ob.N_l[l], T = ob.T_l[l];
  const bool hashed = (ob.hashed_mask >> l) & 1u;
  const float* G = (a.params_override ? a.params_override : ob.params) + ob.off[l];
  for (int k = k0 + threadIdx.x; k < k0 + SPAN; k += blockDim.x) {
    const int64_t ks = (int64_t)bb.blk * RM_SCAT_WG + k;
    if (ks >= bp.n_samples) break;
    const int64_t s = bp.s_begin + ks;
    const RayRec R = a.rays[s / NS];
    if (!ray_active(R.flags)) continue;
    float p[3];
    sample_pos(R, (int)(s % NS), ob.half, p);
    if (!occupied(ob.occ, p)) {  // skipped sample: no gather, zero encoding
      if (a.e_bf16)
        ((uint32_t*)a.e)[(int64_t)l * a.S + s] = 0u;
      else
        a.e[(int64_t)l * a.S + s] = make_float2(0.0f, 0.0f);
      continue;
    }
    Cell cl;
    make_cell(p, N, cl);
    uint32_t idx[8];
    float w[8];
    // on levels where consecutive samples of a ray touch, parity slots: a
    // vertex two lanes share is then loaded by one instruction at one address
    const uint32_t flip = bp.merge ? cell_parity(cl) : 0u;
    cell_corners(cl, N, T, hashed, idx, flip);
    cell_weights(cl, w, flip);
    // The two corners of an x-pair are neighbouring entries on dense levels
    // (index + 1) and, when the cell's x is even, on hashed ones (x enters
    // the hash with factor 1: index ^ 1): then one 16-byte load brings both,
    // halving the cache requests of the pair.
    float2 g[8];
    const bool adj = !hashed || (cl.c[0] & 1u) == 0u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t i0 = idx[2 * q], i1 = idx[2 * q + 1];
      if (adj) {
        const uint32_t lo = i0 < i1 ? i0 : i1;
        const float4 v = *(const float4*)(G + 2 * (int64_t)lo);
        g[2 * q] = i0 == lo ? make_float2(v.x, v.y) : make_float2(v.z, v.w);
        g[2 * q + 1] = i1 == lo ? make_float2(v.x, v.y) : make_float2(v.z, v.w);
      } else {
        g[2 * q] = *(const float2*)(G + 2 * (int64_t)i0);
        g[2 * q + 1] = *(const float2*)(G + 2 * (int64_t)i1);
      }
    }
    float ex = 0.0f, ey = 0.0f;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      ex = fmaf(w[b], g[b].x, ex);
      ey = fmaf(w[b], g[b].y, ey);
    }
    if (a.e_bf16)  // the BF16 MLP reads the encoding rounded to BF16, nothing else
      ((uint32_t*)a.e)[(int64_t)l * a.S + s] = pack_bf16x2(ex, ey);
    else
      a.e[(int64_t)l * a.S + s] = make_float2(ex, ey);
  }
}

// One Adam update of parameter p with gradient g (moments m, v; bias
// corrections bc1, bc2 of the step).
__device__ inline void adam1(float& p, float& m, float& v, float g, const StepArgs& a, float bc1,
                             float bc2) {
  m = a.beta1 * m + (1.0f - a.beta1) * g;
  v = a.beta2 * v + (1.0f - a.beta2) * (g * g);
  p -= a.lr * (m / bc1) / (sqrtf(v / bc2) + a.eps);
}

// Adam on the two features of the table entry at float offset off, with
// gradient (gx, gy); the object's step has been advanced by the pack kernel.
__device__ inline void adam_entry(const ObjStatic& ob, int64_t off, float gx, float gy,
                                  const StepArgs& a, float bc1, float bc2) {
  float2 p = *(float2*)(ob.params + off), m = *(float2*)(ob.m + off), v = *(float2*)(ob.v + off);
  adam1(p.x, m.x, v.x, gx, a, bc1, bc2);
  adam1(p.y, m.y, v.y, gy, a, bc1, bc2);
  *(float2*)(ob.params + off) = p;
  *(float2*)(ob.m + off) = m;
  *(float2*)(ob.v + off) = v;
}

// ---------------------------------------------------------------------------
// K6: encoding backward, grad[idx_b] += w_b * de for the 8 corners of every
// sample, as a binned scatter.  Float atomics on a table cost per cache line
// an instruction touches, and on the fine levels no two samples of a ray
// share a cell, so direct atomics are bound by one line per corner.  Instead
// the (entry, value) records are sorted into regions of RM_RB entries, and
// workgroups per region sum them in LDS and update the region of the
// gradient with coalesced memory operations:
//   k_bin_scatter  per block of samples: rank the records per region, reserve
//                  space in the regions' bins, write them out sorted by region
//                  (a full bin falls back to atomics)
//   k_bin_acc      K workgroups per region: LDS sums, then the gradient
//                  region is updated (plain stores when K = 1 -- the gradient
//                  is zero on entry -- atomics on consecutive entries
//                  otherwise, and read-modify-write if the bin overflowed)
// The bins' fill counters are zeroed by the gather kernel of the same pass.

// A record of the gradient scatter: the two feature values of one corner,
// each rounded to nearest at 17 mantissa bits (a change of at most 2^-18 of
// the value; the sums are then taken to about 2^-38 of an entry's largest
// term), with the entry's index within its region (RM_RB_BITS <= 12 bits) in
// the 6 mantissa bits freed in each.  Zero stays zero, infinities and NaNs
// keep their class.
static_assert(RM_RB_BITS <= 12, "the entry index takes 6 mantissa bits of each value");

__device__ inline uint32_t rec_round(float x) { return (__float_as_uint(x) + 0x20u) & ~0x3Fu; }

__device__ inline float2 rec_pack(float2 v, uint32_t e) {
  return make_float2(__uint_as_float(rec_round(v.x) | (e & 0x3Fu)),
                     __uint_as_float(rec_round(v.y) | ((e >> 6) & 0x3Fu)));
}

__device__ inline uint32_t rec_entry(float x, float y) {
  return (__float_as_uint(x) & 0x3Fu) | ((__float_as_uint(y) & 0x3Fu) << 6);
}

__device__ inline float rec_value(float x) { return __uint_as_float(__float_as_uint(x) & ~0x3Fu); }

// Stores of data that no kernel reads back while it could still be in the
// L2 (gradient records, read by the next kernel after the whole scatter;
// parameters and moments after their Adam update): written past the L2's
// allocation (measured: the accumulation that follows runs 6 % faster).
typedef float rm_f2v __attribute__((ext_vector_type(2)));
__device__ inline void nt_store2(float2* p, float2 v) {
  rm_f2v w;
  w[0] = v.x;
  w[1] = v.y;
  __builtin_nontemporal_store(w, (rm_f2v*)p);
}

// The 8 corner records of sample s at level l of object ob and its cell;
// false (values zero) if none.
template <int NS>
__device__ inline bool bin_records(const StepArgs& a, const ObjStatic& ob, int l, uint32_t N,
                                   uint32_t T, bool hashed, bool par, int64_t s,
                                   uint32_t idx[8], float2 v[8], Cell& cl) {
#pragma unroll
  for (int b = 0; b < 8; ++b) v[b] = make_float2(0.0f, 0.0f);
  // the ray's origin, direction, t_n, delta and flags and the sample's
  // adjoint are loaded together, before either test (one memory round trip)
  const float4* rp = (const float4*)(a.rays + s / NS);
  const float4 r0 = rp[0], r1 = rp[1];
  const uint32_t flags = a.rays[s / NS].flags;
  const float2 g = a.de[(int64_t)l * a.S + s];
  const float half[3] = {ob.half[0], ob.half[1], ob.half[2]};
  asm volatile("" ::"v"(r0.x), "v"(r1.x), "v"(flags), "v"(g.x), "v"(half[0]), "v"(half[1]),
               "v"(half[2]));
  if (!ray_active(flags)) return false;
  if (g.x == 0.0f && g.y == 0.0f) return false;
  RayRec R;
  R.o[0] = r0.x, R.o[1] = r0.y, R.o[2] = r0.z;
  R.d[0] = r0.w, R.d[1] = r1.x, R.d[2] = r1.y;
  R.tn = r1.z, R.delta = r1.w;
  float p[3];
  sample_pos(R, (int)(s % NS), half, p);
  make_cell(p, N, cl);
  const uint32_t flip = par ? cell_parity(cl) : 0u;
  cell_corners(cl, N, T, hashed, idx, flip);
  float w[8];
  cell_weights(cl, w, flip);
#pragma unroll
  for (int b = 0; b < 8; ++b) v[b] = make_float2(w[b] * g.x, w[b] * g.y);
  return true;
}

// Shared corners of consecutive samples.  Cells c and n = c + d share a
// vertex only if |d| <= 1 on every axis; corner b of c (vertex c + bits(b))
// is then a corner of n where d is 0, or where d = +1 and bit b is 1, or
// d = -1 and bit b is 0.
__device__ inline uint32_t shared_corners(int c0, int c1, int c2, int n0, int n1, int n2) {
  const int d0 = n0 - c0, d1 = n1 - c1, d2 = n2 - c2;
  if (abs(d0) > 1 || abs(d1) > 1 || abs(d2) > 1) return 0u;
  const uint32_t m = (uint32_t)(d0 != 0) | ((uint32_t)(d1 != 0) << 1) | ((uint32_t)(d2 != 0) << 2);
  const uint32_t up = (uint32_t)(d0 > 0) | ((uint32_t)(d1 > 0) << 1) | ((uint32_t)(d2 > 0) << 2);
  uint32_t r = 0u;
#pragma unroll
  for (int b = 0; b < 8; ++b) r |= (uint32_t)(((uint32_t)b & m) == up) << b;
  return r;
}

// Parity slots: slot q of a cell holds its corner b = q ^ pc, pc the
// cell's coordinate parities (bit k: c_k & 1), so slot q is the corner whose
// vertex has parities q, and a vertex takes the same slot in every cell it
// is a corner of.  Corner b and corner b ^ 1 stay an x-pair.

// bit b of the result is bit b ^ m of x (8 bits)
__device__ inline uint32_t xor_permute_bits(uint32_t x, uint32_t m) {
  if (m & 1u) x = ((x & 0x55u) << 1) | ((x >> 1) & 0x55u);
  if (m & 2u) x = ((x & 0x33u) << 2) | ((x >> 2) & 0x33u);
  if (m & 4u) x = ((x & 0x0Fu) << 4) | ((x >> 4) & 0x0Fu);
  return x;
}

// the value of lane + O (undefined past the wave's last lane)
template <int O>
__device__ inline int lane_down(int x) {
  if constexpr (O == 1) return dppi<0x130>(x);  // wave_shl:1
  else return __shfl_down(x, O, 64);
}

template <int O>
__device__ inline float lane_down_f(float x) {
  return __int_as_float(lane_down<O>(__float_as_int(x)));
}

// One step of a segmented suffix sum over chains of lanes, in parity slots.
// Bit q of open says that the sum in v[q] covers lanes lane .. lane + O - 1
// of its vertex's chain and the chain goes on; the sum of lane + O (the
// same slot there) is added and the chain's end there carried over.
// Returns false, adding nothing, once no chain of the wave is open.
template <int O>
__device__ inline bool chain_step(float2 v[8], uint32_t& open) {
  if (__ballot(open != 0u) == 0ull) return false;
  float2 y[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) y[q] = make_float2(lane_down_f<O>(v[q].x), lane_down_f<O>(v[q].y));
  const uint32_t yo = (uint32_t)lane_down<O>((int)open);
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if ((open >> q) & 1u) {
      v[q].x += y[q].x;
      v[q].y += y[q].y;
    }
  open &= yo;
  return true;
}

// Exclusive scan of cnt[0..n) into base[0..n) by a whole block of WG
// threads (n <= 8 * WG); returns the total to every thread.
template <int WG>
__device__ inline int block_exclusive_scan(const int* cnt, int* base, int n, int* s_wsum) {
  constexpr int NW = WG / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (n + WG - 1) / WG;  // contiguous entries per thread
  const int j0 = tid * per;
  int mine = 0;
  for (int j = j0; j < j0 + per && j < n; ++j) mine += cnt[j];
  const int inc = wave_incl_prefix_i(mine);
  if (lane == 63) s_wsum[wave] = inc;
  __syncthreads();
  int woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    woff += w < wave ? s_wsum[w] : 0;
    tot += s_wsum[w];
  }
  int run = woff + inc - mine;
  for (int j = j0; j < j0 + per && j < n; ++j) {
    base[j] = run;
    run += cnt[j];
  }
  __syncthreads();
  return tot;
}

// One block: RM_SCAT_WG samples of one (object, level) pair, up to 8 records
// each.  The records are ranked per region in LDS, each region's share of
// the block is reserved in its bin with one global atomic, and the records,
// sorted by region through LDS, are written out with consecutive lanes on
// consecutive slots.  Slots beyond a bin's capacity go to the gradient
// directly (atomics).  The order of records inside a bin depends on timing;
// the fixed-point region sums do not.
template <int NS>
__global__ __launch_bounds__(RM_SCAT_WG) void k_bin_scatter(StepArgs a) {
  // dynamic LDS: staging of the sorted records, then three per-region arrays
  // of a.bin_max_R entries
  extern __shared__ __align__(16) char dyn[];
  float2* s_val = (float2*)dyn;                          // RM_SCAT_WG * 8
  uint32_t* s_id = (uint32_t*)(s_val + RM_SCAT_WG * 8);  // RM_SCAT_WG * 8
  int* lcnt = (int*)(s_id + RM_SCAT_WG * 8);   // records of the block per region
  int* lbase = lcnt + a.bin_max_R;             // their first position in the staging
  int* gpos = lbase + a.bin_max_R;             // first slot reserved in the region's bin
  __shared__ int s_wsum[RM_SCAT_WG / 64];
  // Workgroup i runs on XCD i mod 8: numbered so that each XCD takes a
  // contiguous range of blocks, the blocks of a pair then reserve space in
  // that pair's bins from one XCD and fill them in block order (measured:
  // this kernel 3 % and the accumulation that reads the bins 6 % faster
  // than with consecutive blocks spread over the XCDs).
  const int per_xcd = (a.n_bblocks + 7) >> 3;
  const int jb = (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3);
  if (jb >= a.n_bblocks) return;
  const BinBlock bb = a.bblocks[a.bb_begin + jb];
  const BinPair bp = a.bpairs[bb.pair];
  const int tid = threadIdx.x;
  for (int r = tid; r < bp.R; r += RM_SCAT_WG) lcnt[r] = 0;
  __syncthreads();
  const int64_t k = (int64_t)bb.blk * RM_SCAT_WG + tid;
  uint32_t idx[8];
  float2 v[8];
  int rank[8];
  const ObjStatic& ob = a.objs[a.sobj[bp.so].obj];  // uniform in the block
  const uint32_t NL = ob.N_l[bp.l], TL = ob.T_l[bp.l];
  const bool hashed = (ob.hashed_mask >> bp.l) & 1u;
  float* gl = (a.grad_override ? a.grad_override : ob.grad) + ob.off[bp.l];
  float2* rval = a.rec_val + bp.rec_base;
  Cell cl;
  const bool has = k < bp.n_samples &&
                   bin_records<NS>(a, ob, bp.l, NL, TL, hashed, bp.merge, bp.s_begin + k, idx,
                                   v, cl);
  uint32_t keep = has ? 0xFFu : 0u;  // bit b: corner b is written as a record
  if (bp.merge) {
    // Consecutive samples of a ray (consecutive lanes) share corners where
    // their cells touch, and runs of samples share a whole cell.  A vertex's
    // occurrences along the ray form a chain of lanes linked corner to
    // corner; every chain is summed into its first lane (a segmented suffix
    // sum by doubling, at most 6 steps, in parity slots so that a vertex
    // keeps its slot from lane to lane), which alone writes the record.  A
    // sample without records (a zero adjoint, or skipped by the occupancy
    // test) breaks the chains through it.
    const int lane = tid & 63;
    const int ray = (int)((bp.s_begin + k) / NS);
    const int c0 = has ? (int)cl.c[0] : -2, c1 = has ? (int)cl.c[1] : -2,
              c2 = has ? (int)cl.c[2] : -2;
    // the next lane's values (wave_shl:1), read by every lane of the wave
    const int nh = dppi<0x130>(has ? 1 : 0), nr = dppi<0x130>(ray);
    const int n0 = dppi<0x130>(c0), n1 = dppi<0x130>(c1), n2 = dppi<0x130>(c2);
    const bool next_in = has && lane < 63 && nh != 0 && nr == ray;
    // idx and v are in parity slots (bin_records with par)
    const uint32_t pc = (uint32_t)(c0 & 1) | ((uint32_t)(c1 & 1) << 1) | ((uint32_t)(c2 & 1) << 2);
    uint32_t open = next_in ? xor_permute_bits(shared_corners(c0, c1, c2, n0, n1, n2), pc) : 0u;
    // vertices the previous lane's chains continue into are summed there
    // (wave_shr:1; lane 0 reads 0: no chain comes in)
    keep &= ~(uint32_t)dppi<0x138>((int)open);
    if (chain_step<1>(v, open))
      if (chain_step<2>(v, open))
        if (chain_step<4>(v, open))
          if (chain_step<8>(v, open))
            if (chain_step<16>(v, open)) chain_step<32>(v, open);
  }
  if (keep) {
    // an x-pair of corners in one region takes both ranks with one atomic
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool k0 = (keep >> (2 * q)) & 1u, k1 = (keep >> (2 * q + 1)) & 1u;
      const uint32_t r0 = idx[2 * q] >> RM_RB_BITS, r1 = idx[2 * q + 1] >> RM_RB_BITS;
      if (k0 && k1 && r0 == r1) {
        rank[2 * q] = atomicAdd(&lcnt[r0], 2);
        rank[2 * q + 1] = rank[2 * q] + 1;
      } else {
        if (k0) rank[2 * q] = atomicAdd(&lcnt[r0], 1);
        if (k1) rank[2 * q + 1] = atomicAdd(&lcnt[r1], 1);
      }
    }
  }
  __syncthreads();
  // reserve the block's share of each bin first; with at most one region
  // per thread the reservations are in flight through the scan and the
  // staging (the barriers wait for LDS operations only)
  int mine = 0;
  const bool one = bp.R <= RM_SCAT_WG;
  if (one && tid < bp.R && lcnt[tid]) mine = atomicAdd(&a.bin_count[bp.bin_base + tid], lcnt[tid]);
  if (!one)
    for (int r = tid; r < bp.R; r += RM_SCAT_WG)
      gpos[r] = lcnt[r] ? atomicAdd(&a.bin_count[bp.bin_base + r], lcnt[r]) : 0;
  const int n = block_exclusive_scan<RM_SCAT_WG>(lcnt, lbase, bp.R, s_wsum);
  if (keep) {
    int lb[8];  // all eight bases first: one LDS round trip
#pragma unroll
    for (int b = 0; b < 8; ++b) lb[b] = lbase[idx[b] >> RM_RB_BITS];
#pragma unroll
    for (int b = 0; b < 8; ++b)
      if ((keep >> b) & 1u) {
        const int j = lb[b] + rank[b];
        s_id[j] = idx[b];
        s_val[j] = v[b];
      }
  }
  if (one && tid < bp.R) gpos[tid] = mine;
  __syncthreads();
  // per region: slot of staging position j is dst[r] + j (relative to the
  // pair's records) as long as it stays below the bin's end lim[r]
  int* dst = lbase;  // reused: lbase is read once per region here
  int* lim = gpos;
  for (int r = tid; r < bp.R; r += RM_SCAT_WG) {
    const int b0 = r * bp.cap;
    const int d = b0 + gpos[r] - lbase[r];
    dst[r] = d;
    lim[r] = b0 + bp.cap;
  }
  __syncthreads();
  // four records per thread and round: their LDS reads are issued together
  constexpr int U = 4;
  for (int j0 = tid; j0 < n; j0 += U * RM_SCAT_WG) {
    uint32_t id[U];
    float2 val[U];
    int d[U], lm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * RM_SCAT_WG;
      id[u] = j < n ? s_id[j] : 0u;
      val[u] = j < n ? s_val[j] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = (int)(id[u] >> RM_RB_BITS);
      d[u] = dst[r];
      lm[u] = lim[r];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * RM_SCAT_WG;
      if (j >= n) break;
      const int slot = d[u] + j;
      if (slot < lm[u]) {
        nt_store2(&rval[slot], rec_pack(val[u], id[u] & (RM_RB - 1)));
      } else {  // bin full: direct atomics (correct, only slower)
        unsafeAtomicAdd(gl + 2 * (int64_t)id[u], val[u].x);
        unsafeAtomicAdd(gl + 2 * (int64_t)id[u] + 1, val[u].y);
      }
    }
  }
}

// Region sums are taken in LDS as 64-bit fixed point: float atomics in LDS
// run about 24 times slower than integer ones on this chip.  A first pass
// takes, per entry, the largest binary exponent of its records (an integer
// max); the second adds every record scaled by 2^(RM_FX_BITS - that
// exponent), rounded to an integer (|term| < 2^(RM_FX_BITS + 1)), so each
// term is kept to 2^-RM_FX_BITS of the entry's largest one -- finer than an
// FP32 rounding of the sum -- and the sum is exact and independent of order.
// Up to 2^(62 - RM_FX_BITS) records per entry and workgroup fit.

// biased FP32 exponent field of |v| (0 for zero and subnormals)
__device__ inline uint32_t exp_field(float v) { return (__float_as_uint(v) >> 23) & 0xffu; }

// 2^k as a double, k within the normal range
__device__ inline double pow2d(int k) { return __longlong_as_double((long long)(k + 1023) << 52); }

__device__ inline void fx_add(unsigned long long* acc, const uint32_t* emax, uint32_t e, float vx,
                              float vy) {
  const uint32_t eb = emax[e] > 1u ? emax[e] : 1u;
  const double sc = pow2d(RM_FX_BITS + 127 - (int)eb);  // |v| < 2^(eb - 126)
  atomicAdd(&acc[2 * e], (unsigned long long)__double2ll_rn((double)vx * sc));
  atomicAdd(&acc[2 * e + 1], (unsigned long long)__double2ll_rn((double)vy * sc));
}

__device__ inline void rec_max(uint32_t* emax, float x, float y) {
  atomicMax(&emax[rec_entry(x, y)], max(exp_field(x), exp_field(y)));
}

__device__ inline void rec_add(unsigned long long* acc, const uint32_t* emax, float x, float y) {
  fx_add(acc, emax, rec_entry(x, y), rec_value(x), rec_value(y));
}

__global__ __launch_bounds__(RM_ACC_WG) void k_bin_acc(StepArgs a) {
  __shared__ uint32_t emax[RM_RB];
  __shared__ unsigned long long acc[2 * RM_RB];
  const Bin bn = a.bins[a.bin_begin + blockIdx.x];
  const BinPair bp = a.bpairs[bn.pair];
  int n = a.bin_count[bp.bin_base + bn.region];
  const bool spilled = n > bp.cap;  // some records went to the gradient directly
  n = spilled ? bp.cap : n;
  // this workgroup's share of the bin: [i0, i1), multiples of 4 but the end
  const int per = ((n + bp.K - 1) / bp.K + 3) & ~3;
  const int i0 = bn.k * per;
  const int i1 = (i0 + per < n) ? i0 + per : n;
  // The sole workgroup of a region (K = 1) applies a training step's Adam
  // update to all of the region's entries, even with no records; shared
  // regions are finished by k_bin_finish.
  const bool adam_here = a.fuse_adam && bp.K == 1;
  if (i0 >= i1 && !adam_here) return;  // empty share: nothing to add
  const int oi = a.sobj[bp.so].obj;
  const ObjStatic& ob = a.objs[oi];
  // entries of this region (a dense level's last region is partial)
  const int64_t e0 = (int64_t)bn.region * RM_RB;
  const int64_t rem = (int64_t)ob.T_l[bp.l] - e0;
  const int ne = rem < RM_RB ? (int)rem : RM_RB;
  const int64_t off0 = ob.off[bp.l] + 2 * e0;  // float offset of the region
  // Adam operands of this thread's entries, loaded now so that they arrive
  // while the records are summed
  constexpr int EPT = RM_RB / RM_ACC_WG;
  float2* __restrict__ Pp = (float2*)(ob.params + off0);
  float2* __restrict__ Pm = (float2*)(ob.m + off0);
  float2* __restrict__ Pv = (float2*)(ob.v + off0);
  float2 ap[EPT], am[EPT], av[EPT];
  if (adam_here) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = threadIdx.x + k * RM_ACC_WG;
      if (e < ne) {
        ap[k] = Pp[e];
        am[k] = Pm[e];
        av[k] = Pv[e];
      }
    }
  }
  for (int e = threadIdx.x; e < RM_RB; e += RM_ACC_WG) {
    emax[e] = 0u;
    acc[2 * e] = 0ull;
    acc[2 * e + 1] = 0ull;
  }
  __syncthreads();
  const int64_t base = bp.rec_base + (int64_t)bn.region * bp.cap;  // multiple of 4
  const float4* rv = (const float4*)(a.rec_val + base);  // two records per float4
  const int q0 = i0 >> 2, q1 = i1 >> 2;
  // The first RM_ACC_RQ quads of records of each thread stay in registers
  // from the first pass to the second: a share of up to RM_ACC_RQ * 4 *
  // RM_ACC_WG records is read once (the shares of all workgroups in flight
  // do not fit in the L2 between the passes).
  constexpr int RQ = RM_ACC_RQ;
  float4 ca[RQ], cb[RQ];
#pragma unroll
  for (int i = 0; i < RQ; ++i) {
    const int q = q0 + threadIdx.x + i * RM_ACC_WG;
    if (q < q1) {
      ca[i] = rv[2 * q];
      cb[i] = rv[2 * q + 1];
    }
  }
  // pass 1: largest exponent per entry
#pragma unroll
  for (int i = 0; i < RQ; ++i) {
    if (q0 + (int)threadIdx.x + i * RM_ACC_WG < q1) {
      rec_max(emax, ca[i].x, ca[i].y);
      rec_max(emax, ca[i].z, ca[i].w);
      rec_max(emax, cb[i].x, cb[i].y);
      rec_max(emax, cb[i].z, cb[i].w);
    }
  }
  for (int q = q0 + threadIdx.x + RQ * RM_ACC_WG; q < q1; q += RM_ACC_WG) {  // 4 records per lane
    const float4 va = rv[2 * q], vb = rv[2 * q + 1];
    rec_max(emax, va.x, va.y);
    rec_max(emax, va.z, va.w);
    rec_max(emax, vb.x, vb.y);
    rec_max(emax, vb.z, vb.w);
  }
  for (int i = (q1 << 2) + threadIdx.x; i < i1; i += RM_ACC_WG) {  // tail
    const float2 v = a.rec_val[base + i];
    rec_max(emax, v.x, v.y);
  }
  __syncthreads();
  // pass 2: fixed-point sums (records beyond the registers are read again)
#pragma unroll
  for (int i = 0; i < RQ; ++i) {
    if (q0 + (int)threadIdx.x + i * RM_ACC_WG < q1) {
      rec_add(acc, emax, ca[i].x, ca[i].y);
      rec_add(acc, emax, ca[i].z, ca[i].w);
      rec_add(acc, emax, cb[i].x, cb[i].y);
      rec_add(acc, emax, cb[i].z, cb[i].w);
    }
  }
  for (int q = q0 + threadIdx.x + RQ * RM_ACC_WG; q < q1; q += RM_ACC_WG) {
    const float4 va = rv[2 * q], vb = rv[2 * q + 1];
    rec_add(acc, emax, va.x, va.y);
    rec_add(acc, emax, va.z, va.w);
    rec_add(acc, emax, vb.x, vb.y);
    rec_add(acc, emax, vb.z, vb.w);
  }
  for (int i = (q1 << 2) + threadIdx.x; i < i1; i += RM_ACC_WG) {
    const float2 v = a.rec_val[base + i];
    rec_add(acc, emax, v.x, v.y);
  }
  __syncthreads();
  float2* g = (float2*)((a.grad_override ? a.grad_override : ob.grad) + off0);
  const float bc1 = a.state[oi].bc1, bc2 = a.state[oi].bc2;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = threadIdx.x + k * RM_ACC_WG;
    if (e >= ne) break;
    const uint32_t em = emax[e];
    const long long sx = (long long)acc[2 * e], sy = (long long)acc[2 * e + 1];
    float dx = 0.0f, dy = 0.0f;
    if (em == 0xffu) {  // an Inf or NaN among the records
      dx = dy = __int_as_float(0x7fc00000);
    } else if (sx != 0 || sy != 0) {
      const double isc = pow2d((int)(em > 1u ? em : 1u) - 127 - RM_FX_BITS);
      dx = (float)((double)sx * isc);
      dy = (float)((double)sy * isc);
    }
    if (adam_here) {  // the entry's gradient is complete: update, keep g zero
      if (spilled) {
        const float2 x = g[e];
        dx += x.x;
        dy += x.y;
        g[e] = make_float2(0.0f, 0.0f);
      }
      adam1(ap[k].x, am[k].x, av[k].x, dx, a, bc1, bc2);
      adam1(ap[k].y, am[k].y, av[k].y, dy, a, bc1, bc2);
      nt_store2(&Pp[e], ap[k]);
      nt_store2(&Pm[e], am[k]);
      nt_store2(&Pv[e], av[k]);
      continue;
    }
    if (em == 0u && sx == 0 && sy == 0) continue;  // untouched (or only zeros)
    if (bp.K == 1 && !spilled) {  // sole writer of a zero region: plain stores
      g[e] = make_float2(dx, dy);
    } else if (bp.K == 1) {  // the scatter's overflow atomics are in the region too
      float2 x = g[e];
      x.x += dx;
      x.y += dy;
      g[e] = x;
    } else {  // shared region: atomics on consecutive entries
      unsafeAtomicAdd(&g[e].x, dx);
      unsafeAtomicAdd(&g[e].y, dy);
    }
  }
}

// Training steps: Adam on the entries of regions that several workgroups
// summed into the gradient (and leaves it zero for the next step).
__global__ __launch_bounds__(RM_FIN_WG) void k_bin_finish(StepArgs a) {
  const Fin f = a.fins[blockIdx.x];
  const BinPair bp = a.bpairs[f.pair];
  const int oi = a.sobj[bp.so].obj;
  const ObjStatic& ob = a.objs[oi];
  const int64_t e0 = (int64_t)f.region * RM_RB;
  const int64_t rem = (int64_t)ob.T_l[bp.l] - e0;
  const int ne = rem < RM_RB ? (int)rem : RM_RB;
  const int e = f.sub * RM_FIN_WG + threadIdx.x;
  if (e >= ne) return;
  const int64_t off = ob.off[bp.l] + 2 * (e0 + e);
  float2* g = (float2*)(ob.grad + off);
  const float2 x = *g;
  *g = make_float2(0.0f, 0.0f);
  adam_entry(ob, off, x.x, x.y, a, a.state[oi].bc1, a.state[oi].bc2);
}

// ---------------------------------------------------------------------------
// K3: MLP weights -> MFMA operand images.  For a GEMM Out(M x 16 samples) =
// A(M x K) X(K x 16), operand element (t, q, r, lane) is
// A[16t + lane%16][16q + 4(lane/16) + r]; the FP32 image orders it
// ((t Q + q) 4 + r) 64 + lane (one 16x16x4 operand per 64 contiguous values),
// the BF16 image ((t Q + q) 64 + lane) 4 + r (one 16x16x16 operand per lane)
// when K = 16, and for K a multiple of 32 ((t C + c) 64 + lane) 8 + q8 with
// A[16t + lane%16][32c + (q8 < 4 ? 4g + q8 : 16 + 4g + q8 - 4)], g = lane/16
// (one 16x16x32 operand per lane, in the slot order of Mma<1>).
// Operands 8 + 2(k-1) and 9 + 2(k-1) are the k-th hidden-to-hidden matrix of
// a deeper density MLP (nh hidden layers) and its transpose.
__device__ inline float mlp_A(const float* W, int din, int nh, int gemm, int m, int k) {
  const float* W1 = W;
  const float* Wh = W1 + RM_HIDDEN * din;
  const float* W2 = Wh + (nh - 1) * RM_HH;
  const float* W3 = W2 + RM_DOUT * RM_HIDDEN;
  const float* W4 = W3 + RM_HIDDEN * RM_GEO;
  switch (gemm) {
    case 0: return k < din ? W1[m * din + k] : 0.0f;                 // F1 64 x K1
    case 1: return W2[m * RM_HIDDEN + k];                             // F2 16 x 64
    case 2: return k >= 1 ? W3[m * RM_GEO + (k - 1)] : 0.0f;          // F3 64 x 16
    case 3: return m < 3 ? W4[m * RM_HIDDEN + k] : 0.0f;              // F4 16 x 64
    case 4: return k < 3 ? W4[k * RM_HIDDEN + m] : 0.0f;              // B4 64 x 16
    case 5: return m >= 1 ? W3[k * RM_GEO + (m - 1)] : 0.0f;          // B3 16 x 64
    case 6: return W2[k * RM_HIDDEN + m];                             // B2 64 x 16
    case 7: return m < din ? W1[k * din + m] : 0.0f;                  // B1 K1 x 64
    default: {
      const float* H = Wh + ((gemm - 8) >> 1) * RM_HH;
      return (gemm & 1) ? H[k * RM_HIDDEN + m] : H[m * RM_HIDDEN + k];  // Wh_k^T, Wh_k
    }
  }
}

// Also advances each object's Adam step (training steps only): after the ray
// draw, which uses the step as its counter, and before any Adam update.
__global__ __launch_bounds__(256) void k_pack(StepArgs a, int K1) {
  const StepObj so = a.sobj[blockIdx.x];
  const ObjStatic& ob = a.objs[so.obj];
  if (a.fuse_adam && blockIdx.y == 0 && threadIdx.x == 0) {
    ObjState* st = a.state + so.obj;
    const int kk = st->step + 1;
    st->step = kk;
    st->bc1 = (float)(1.0 - pow((double)a.beta1, (double)kk));
    st->bc2 = (float)(1.0 - pow((double)a.beta2, (double)kk));
  }
  const float* W = (a.params_override ? a.params_override : ob.params) + ob.P_grid;
  const int din = ob.din, nh = a.mlp_layers;
  const int Ms[8] = {64, 16, 64, 16, 64, 16, 64, K1};
  const int Ks[8] = {K1, 64, 16, 64, 16, 64, 16, 64};
  const int offs[8] = {RM_OFF_F1, RM_OFF_F2, RM_OFF_F3, RM_OFF_F4,
                       RM_OFF_B4, RM_OFF_B3, RM_OFF_B2, RM_OFF_B1};
  const int64_t stride = RM_WPACK_NH(nh);
  float* o32 = a.wpack32 + (int64_t)blockIdx.x * stride;
  uint16_t* o16 = a.wpack16 + (int64_t)blockIdx.x * stride;
  {  // one operand per block
    const int gm = blockIdx.y;
    const int M = gm < 8 ? Ms[gm] : RM_HIDDEN, K = gm < 8 ? Ks[gm] : RM_HIDDEN, Q = K / 16;
    const int off = gm < 8 ? offs[gm] : RM_OFF_HF(1) + (gm - 8) * RM_HH;
    for (int j = threadIdx.x; j < M * K; j += blockDim.x) {
      {  // FP32 image
        const int lane = j & 63, r = (j >> 6) & 3, tq = j >> 8;
        const int q = tq % Q, t = tq / Q;
        o32[off + j] = mlp_A(W, din, nh, gm, 16 * t + (lane & 15), 16 * q + 4 * (lane >> 4) + r);
      }
      if (K % 32 == 0) {  // BF16 image of a 16x16x32 operand (slot order of Mma<1>)
        const int q8 = j & 7, lane = (j >> 3) & 63, tc = j >> 9, C = K / 32;
        const int c = tc % C, t = tc / C, g = lane >> 4;
        const int col = 32 * c + (q8 < 4 ? 4 * g + q8 : 16 + 4 * g + (q8 - 4));
        o16[off + j] = f2bf(mlp_A(W, din, nh, gm, 16 * t + (lane & 15), col));
      } else {  // BF16 image of a 16x16x16 operand
        const int r = j & 3, lane = (j >> 2) & 63, tq = j >> 8;
        const int q = tq % Q, t = tq / Q;
        o16[off + j] =
            f2bf(mlp_A(W, din, nh, gm, 16 * t + (lane & 15), 16 * q + 4 * (lane >> 4) + r));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K4: fused per-ray field kernel.
//
// A wave owns one ray at a time; its N samples are processed in blocks of 16.
// Activations are kept transposed, [feature][sample], as 16x16 MFMA result
// fragments (lane = sample column, 4 feature rows per lane), which are
// directly the B operands of the next layer: every forward and input-adjoint
// GEMM chains in registers.  Weight gradients contract over samples and need
// the [feature][sample] tiles in LDS (per-wave staging).
//
// PREC 0: FP32 MFMA 16x16x4.  PREC 1: BF16 MFMA 16x16x16, FP32 accumulation.
template <int PREC>
struct Mma;

template <>
struct Mma<0> {
  typedef float wtype;
  static constexpr int STRIDE = 17;  // staging row stride (floats)
  template <int M, int K>
  __device__ static inline void gemm(const float* wA, const floatx4* X, floatx4* Out, int lane) {
    constexpr int Q = K / 16;
#pragma unroll
    for (int t = 0; t < M / 16; ++t) {
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wA[((t * Q + q) * 4 + r) * 64 + lane],
                                                    X[q][r], acc, 0, 0, 0);
      }
      Out[t] = acc;
    }
  }
  __device__ static inline void stage(float* buf, const floatx4* F, int nf, int lane) {
    const int g = lane >> 4, n = lane & 15;
    for (int f = 0; f < nf; ++f) {
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[(16 * f + 4 * g + r) * STRIDE + n] = F[f][r];
    }
  }
  // acc[t][u] += G^T(16t.., 16 samples) X(16 samples, 16u..)
  template <int MG, int MX>
  __device__ static inline void dw(const float* gb, const float* xb, floatx4* acc, int lane) {
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < MG / 16; ++t)
#pragma unroll
      for (int u = 0; u < MX / 16; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[t * (MX / 16) + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              gb[(16 * t + i) * STRIDE + 4 * c + g], xb[(16 * u + i) * STRIDE + 4 * c + g],
              acc[t * (MX / 16) + u], 0, 0, 0);
  }
};

__device__ inline bf16x4_t cvt_bf16x4(floatx4 v) { return __builtin_convertvector(v, bf16x4_t); }

// PREC 1 operands.  A contraction over K >= 32 runs as 16x16x32 MFMAs whose K
// slots are ordered so that two consecutive [feature][sample] result
// fragments (features 32c..32c+15 and 32c+16..32c+31) are, concatenated per
// lane, its B operand: lane (g, n) feeds slots 8g..8g+7 = features
// 32c + 4g + 0..3 and 32c + 16 + 4g + 0..3 of sample n; the weight image
// holds A in the same slot order (k_pack).  K = 16 runs as 16x16x16.
template <>
struct Mma<1> {
  typedef uint16_t wtype;
  static constexpr int STRIDE = 20;  // staging row stride (bf16), keeps 8-byte alignment
  // Out(M x 16 samples) = A(M x K) X(K x 16), X given as BF16 fragments
  template <int M, int K>
  __device__ static inline void gemm_b(const uint16_t* wA, const bf16x4_t* xb, floatx4* Out,
                                       int lane) {
    if constexpr (K % 32 == 0) {
      constexpr int C = K / 32;
      bf16x8_t x8[C];
#pragma unroll
      for (int c = 0; c < C; ++c)
        x8[c] = __builtin_shufflevector(xb[2 * c], xb[2 * c + 1], 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
      for (int t = 0; t < M / 16; ++t) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const bf16x8_t av = *(const bf16x8_t*)(wA + ((t * C + c) * 64 + lane) * 8);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, x8[c], acc, 0, 0, 0);
        }
        Out[t] = acc;
      }
    } else {
      constexpr int Q = K / 16;
#pragma unroll
      for (int t = 0; t < M / 16; ++t) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const shortx4 av = *(const shortx4*)(wA + ((t * Q + q) * 64 + lane) * 4);
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
              av, __builtin_bit_cast(shortx4, xb[q]), acc, 0, 0, 0);
        }
        Out[t] = acc;
      }
    }
  }
  template <int M, int K>
  __device__ static inline void gemm(const uint16_t* wA, const floatx4* X, floatx4* Out,
                                     int lane) {
    bf16x4_t xb[K / 16];
#pragma unroll
    for (int q = 0; q < K / 16; ++q) xb[q] = cvt_bf16x4(X[q]);
    gemm_b<M, K>(wA, xb, Out, lane);
  }
  __device__ static inline void stage_b(uint16_t* buf, const bf16x4_t* F, int nf, int lane) {
    const int g = lane >> 4, n = lane & 15;
    for (int f = 0; f < nf; ++f) {
      const shortx4 v = __builtin_bit_cast(shortx4, F[f]);
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[(16 * f + 4 * g + r) * STRIDE + n] = (uint16_t)v[r];
    }
  }
  __device__ static inline void stage(uint16_t* buf, const floatx4* F, int nf, int lane) {
    const int g = lane >> 4, n = lane & 15;
    for (int f = 0; f < nf; ++f) {
      const shortx4 v = __builtin_bit_cast(shortx4, cvt_bf16x4(F[f]));
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[(16 * f + 4 * g + r) * STRIDE + n] = (uint16_t)v[r];
    }
  }
  template <int MG, int MX>
  __device__ static inline void dw(const uint16_t* gb, const uint16_t* xb, floatx4* acc,
                                   int lane) {
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < MG / 16; ++t) {
      const shortx4 av = *(const shortx4*)(gb + (16 * t + i) * STRIDE + 4 * g);
#pragma unroll
      for (int u = 0; u < MX / 16; ++u) {
        const shortx4 bv = *(const shortx4*)(xb + (16 * u + i) * STRIDE + 4 * g);
        acc[t * (MX / 16) + u] =
            __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t * (MX / 16) + u], 0, 0, 0);
      }
    }
  }
  // Tiles of 32 samples (two 16-sample blocks side by side): rows of
  // STRIDE2 values, 16-byte aligned, so a lane reads 8 consecutive samples.
  static constexpr int STRIDE2 = 40;
  __device__ static inline void stage_b2(uint16_t* buf, const bf16x4_t* F, int nf, int lane,
                                         int col0) {
    const int g = lane >> 4, n = lane & 15;
    for (int f = 0; f < nf; ++f) {
      const shortx4 v = __builtin_bit_cast(shortx4, F[f]);
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[(16 * f + 4 * g + r) * STRIDE2 + col0 + n] = (uint16_t)v[r];
    }
  }
  // dW += G X^T over 32 samples, one 16x16x32 MFMA per output tile: lane
  // (i, g) holds samples 8g .. 8g+7 of row i of both operands (the same
  // order of the contracted index on both sides)
  template <int MG, int MX>
  __device__ static inline void dw32(const uint16_t* gb, const uint16_t* xb, floatx4* acc,
                                     int lane) {
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < MG / 16; ++t) {
      const bf16x8_t av = *(const bf16x8_t*)(gb + (16 * t + i) * STRIDE2 + 8 * g);
#pragma unroll
      for (int u = 0; u < MX / 16; ++u) {
        const bf16x8_t bv = *(const bf16x8_t*)(xb + (16 * u + i) * STRIDE2 + 8 * g);
        acc[t * (MX / 16) + u] =
            __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t * (MX / 16) + u], 0, 0, 0);
      }
    }
  }
};

// ReLU of FP32 pre-activations, rounded to BF16: rounding to nearest
// commutes with max(x, 0), and a BF16 value read as int16 is negative exactly
// when its sign bit is set, so one packed 16-bit integer max does two units.
__device__ inline bf16x4_t relu_b(floatx4 x) {
  const shortx4 v = __builtin_bit_cast(shortx4, cvt_bf16x4(x));
  const shortx4 z = {0, 0, 0, 0};
  return __builtin_bit_cast(bf16x4_t, __builtin_elementwise_max(v, z));
}

// An FP32 adjoint rounded to BF16 and kept where the unit's ReLU output h
// (BF16, >= 0) is positive: min(h, 1) * 0xFFFF as 16-bit lanes is the mask.
// (op_sel_hi:[1,0]: the high lane also reads the constant's low half, which
// is where an inline constant of a packed instruction sits.)
__device__ inline bf16x4_t mask_b(floatx4 d, bf16x4_t h) {
  const uint2 hb = __builtin_bit_cast(uint2, h);
  uint32_t m0, m1;
  asm("v_pk_min_u16 %0, %1, 1 op_sel_hi:[1,0]" : "=v"(m0) : "v"(hb.x));
  asm("v_pk_min_u16 %0, %1, 1 op_sel_hi:[1,0]" : "=v"(m1) : "v"(hb.y));
  asm("v_pk_mul_lo_u16 %0, %1, -1 op_sel_hi:[1,0]" : "=v"(m0) : "v"(m0));
  asm("v_pk_mul_lo_u16 %0, %1, -1 op_sel_hi:[1,0]" : "=v"(m1) : "v"(m1));
  const uint2 db = __builtin_bit_cast(uint2, cvt_bf16x4(d));
  return __builtin_bit_cast(bf16x4_t, make_uint2(db.x & m0, db.y & m1));
}

__device__ inline void relu4(floatx4* F, int n) {
  for (int f = 0; f < n; ++f) {
#pragma unroll
    for (int r = 0; r < 4; ++r) F[f][r] = F[f][r] > 0.0f ? F[f][r] : 0.0f;
  }
}

__device__ inline float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }

// Loads the encoding of 16 samples (s0 .. s0+15) as K1/16 fragments:
// fragment q, register r, lane (g, n) = feature 16q + 4g + r of sample s0 + n,
// feature f = level f/2, component f%2 of the [L][S] float2 buffer.
template <int K1>
__device__ inline void load_e(const float2* e, int64_t S, int64_t s, int L, int g, floatx4* E) {
#pragma unroll
  for (int q = 0; q < K1 / 16; ++q) {
    const int l0 = 8 * q + 2 * g, l1 = l0 + 1;
    const float2 v0 = l0 < L ? e[(int64_t)l0 * S + s] : make_float2(0.0f, 0.0f);
    const float2 v1 = l1 < L ? e[(int64_t)l1 * S + s] : make_float2(0.0f, 0.0f);
    E[q][0] = v0.x;
    E[q][1] = v0.y;
    E[q][2] = v1.x;
    E[q][3] = v1.y;
  }
}

// The same fragments from the BF16 pairs of an e_bf16 buffer (bits as stored).
template <int K1>
__device__ inline void load_e_b(const uint32_t* e, int64_t S, int64_t s, int L, int g,
                                bf16x4_t* E) {
#pragma unroll
  for (int q = 0; q < K1 / 16; ++q) {
    const int l0 = 8 * q + 2 * g, l1 = l0 + 1;
    const uint32_t v0 = l0 < L ? e[(int64_t)l0 * S + s] : 0u;
    const uint32_t v1 = l1 < L ? e[(int64_t)l1 * S + s] : 0u;
    E[q] = __builtin_bit_cast(bf16x4_t, (uint64_t)v0 | ((uint64_t)v1 << 32));
  }
}

// NH: hidden layers of the density MLP (1, or 2 and 3 for the model-size
// study); the deeper variants run one wave per SIMD (their 64 x 64 weight
// gradients are accumulated in registers), and their work-item record shares
// LDS with the weights, which are no longer read when it is written.
template <int PREC, int NS, int K1, int NH>
#ifndef RM_FIELD_BF16_WAVES
#define RM_FIELD_BF16_WAVES 2
#endif
__global__ __launch_bounds__(RM_WG) __attribute__((amdgpu_waves_per_eu(NH > 1 ? 1 : (PREC == 1 ? RM_FIELD_BF16_WAVES : 2)))) void k_field(StepArgs a) {
  typedef Mma<PREC> MM;
  typedef typename MM::wtype wt;
  constexpr int NB = NS / 16;             // 16-sample blocks per ray
  constexpr int SPL = NS > 64 ? NS / 64 : 1;  // samples per lane in the composite
  constexpr int STG = 64 * MM::STRIDE;    // one staging tile (64 feature rows)
  constexpr int KQ = K1 / 16;
  // a ray's encodings stay in registers from the forward to the backward
  // pass when they fit (NS <= 64, one hidden layer), else the backward reads
  // them again
  constexpr bool KEEP_E = NH == 1 && NB * KQ <= 8 && (PREC == 0 || RM_FIELD_BF16_WAVES < 3);
  constexpr int NBK = KEEP_E ? NB : 1;
  constexpr int WP = RM_WPACK_NH(NH);
  constexpr int RL = RM_REC_LOSS_NH(NH);
  constexpr int WBYTES = WP * (int)sizeof(wt), RBYTES = (RL + 1) * 4;
  // the work-item record shares LDS with the weights, which are no longer
  // read when it is written (fewer bytes per workgroup, more workgroups per CU)
  constexpr bool ALIAS = NH > 1 || PREC == 1;
  // BF16 with one hidden layer: activations kept as rounded BF16 pairs
  constexpr bool PACKED = PREC == 1 && NH == 1;

  __shared__ __align__(16) char s_wraw[ALIAS && RBYTES > WBYTES ? RBYTES : WBYTES];
  // BF16 with one hidden layer stages tiles of 32 samples (pairs of blocks)
  constexpr int STGS = PACKED ? 64 * Mma<1>::STRIDE2 : STG;
  __shared__ __align__(16) wt s_stage[4][2][STGS];
  __shared__ __align__(16) float s_rv[4][NS * 4];
  __shared__ float s_rec_own[ALIAS ? 1 : RL + 1];
  wt* s_w = (wt*)s_wraw;
  float* s_rec = ALIAS ? (float*)s_wraw : s_rec_own;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n = lane & 15;
  const Item it = a.items[blockIdx.x];
  const StepObj so = a.sobj[it.so];
  const ObjStatic& ob = a.objs[so.obj];
  const int L = ob.L, din = ob.din;
  const int64_t S = a.S;
  const float invB = 1.0f / (float)so.n_rays;
  const int mode = a.mode;

  {  // weights of this object into LDS (16-byte copies)
    const uint4* src = (const uint4*)((PREC ? (const void*)(a.wpack16 + (int64_t)it.so * WP)
                                            : (const void*)(a.wpack32 + (int64_t)it.so * WP)));
    uint4* dst = (uint4*)s_w;
    constexpr int NV = WP * (int)sizeof(wt) / 16;
    for (int j = tid; j < NV; j += RM_WG) dst[j] = src[j];
  }
  __syncthreads();

  const wt* wF1 = s_w + RM_OFF_F1;
  const wt* wF2 = s_w + RM_OFF_F2;
  const wt* wF3 = s_w + RM_OFF_F3;
  const wt* wF4 = s_w + RM_OFF_F4;
  const wt* wB4 = s_w + RM_OFF_B4;
  const wt* wB3 = s_w + RM_OFF_B3;
  const wt* wB2 = s_w + RM_OFF_B2;
  const wt* wB1 = s_w + RM_OFF_B1;
  wt* gbuf = s_stage[wave][0];
  wt* xbuf = s_stage[wave][1];
  float* rv = s_rv[wave];
  // encodings: FP32 fragments, or with the BF16 MLP the stored BF16 pairs as
  // they are (the MLP reads nothing else of them)
  typedef typename std::conditional<PREC == 1, bf16x4_t, floatx4>::type etype;
  auto load_enc = [&](int64_t s, etype* E) {
    if constexpr (PREC == 1)
      load_e_b<K1>((const uint32_t*)a.e, S, s, L, g, E);
    else
      load_e<K1>(a.e, S, s, L, g, E);
  };
  auto gemm_e = [&](const etype* E, floatx4* H) {
    if constexpr (PREC == 1)
      MM::template gemm_b<64, K1>(wF1, E, H, lane);
    else
      MM::template gemm<64, K1>(wF1, E, H, lane);
  };

  floatx4 acc1[4 * KQ], acc2[4], acc3[4], acc4[4];
  floatx4 accH[NH > 1 ? NH - 1 : 1][16];  // hidden-to-hidden weight gradients
#pragma unroll
  for (int j = 0; j < 4 * KQ; ++j) acc1[j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < (NH > 1 ? NH - 1 : 1); ++k)
#pragma unroll
    for (int j = 0; j < 16; ++j) accH[k][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    acc2[j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    acc3[j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    acc4[j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  float loss_w = 0.0f;

  for (int rr = wave; rr < it.n_rays; rr += 4) {
    const int ray = __builtin_amdgcn_readfirstlane(it.ray_begin + rr);
    const RayRec R = a.rays[ray];
    if (!ray_active(R.flags)) {
      if (mode == RM_MODE_FORWARD && lane == 0) {
        if (a.out_rgb) a.out_rgb[3 * ray] = a.out_rgb[3 * ray + 1] = a.out_rgb[3 * ray + 2] = 0.0f;
        if (a.out_depth) a.out_depth[ray] = 0.0f;
        if (a.out_tend) a.out_tend[ray] = 1.0f;
      }
      continue;
    }
    const int64_t sray = (int64_t)ray * NS;

    // ---- forward: sigma, colour of every sample ----
    etype EK[NBK][KQ];
#pragma unroll(KEEP_E ? NB : 1)
    for (int b = 0; b < NB; ++b) {
      etype E[KQ];
      floatx4 H1[4], Y[1], H2[4], Z[1];
      load_enc(sray + 16 * b + n, E);
      if (KEEP_E) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) EK[KEEP_E ? b : 0][q] = E[q];
      }
      if constexpr (PACKED) {  // activations as rounded BF16 pairs
        bf16x4_t H1b[4], Yb[1], H2b[4];
        gemm_e(E, H1);
#pragma unroll
        for (int f = 0; f < 4; ++f) H1b[f] = relu_b(H1[f]);
        MM::template gemm_b<16, 64>(wF2, H1b, Y, lane);
        Yb[0] = cvt_bf16x4(Y[0]);
        MM::template gemm_b<64, 16>(wF3, Yb, H2, lane);
#pragma unroll
        for (int f = 0; f < 4; ++f) H2b[f] = relu_b(H2[f]);
        MM::template gemm_b<16, 64>(wF4, H2b, Z, lane);
      } else {
        gemm_e(E, H1);
        relu4(H1, 4);
#pragma unroll
        for (int k = 1; k < NH; ++k) {  // deeper density MLP: H1 <- ReLU(Wh_k H1)
          floatx4 Hn[4];
          MM::template gemm<64, 64>(s_w + RM_OFF_HF(k), H1, Hn, lane);
          relu4(Hn, 4);
#pragma unroll
          for (int f = 0; f < 4; ++f) H1[f] = Hn[f];
        }
        MM::template gemm<16, 64>(wF2, H1, Y, lane);
        MM::template gemm<64, 16>(wF3, Y, H2, lane);
        relu4(H2, 4);
        MM::template gemm<16, 64>(wF4, H2, Z, lane);
      }
      if (g == 0) {
        float* q = rv + (16 * b + n) * 4;
        q[0] = Y[0][0];
        q[1] = Z[0][0];  // colour logits: the adjoint needs sigmoid(-z) as well
        q[2] = Z[0][1];
        q[3] = Z[0][2];
      }
    }
    wave_lds_sync();

    // ---- volume rendering (Eq. 6) and its adjoint; lane = sample ----
    {
      const uint32_t cls = R.flags & RM_F_CLS;
      const bool bg = (mode == RM_MODE_TRAIN) && cls == RM_CLS_BACKGROUND;
      const bool valid = lane * SPL < NS;
      float y0[SPL], c[SPL][3], zc[SPL][3], sig[SPL], tau[SPL], dist[SPL], w[SPL], Sx[SPL];
      float lane_tau = 0.0f, lane_sig = 0.0f;
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        const int i = lane * SPL + j;
        if (valid) {
          const float* q = rv + i * 4;
          y0[j] = q[0];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            zc[j][k] = q[1 + k];
            c[j][k] = sigmoidf_(zc[j][k]);
          }
          bool live = true;
          if (ob.occ) {
            float p[3];
            sample_pos(R, i, ob.half, p);
            live = occupied(ob.occ, p);
          }
          sig[j] = live ? expf(fminf(y0[j], 15.0f)) : 0.0f;
          if (!live) y0[j] = 16.0f;  // no density adjoint either
          tau[j] = sig[j] * R.delta;
          dist[j] = R.tn + ((float)i + 0.5f) * R.delta;
        } else {
          y0[j] = 0.0f;
          c[j][0] = c[j][1] = c[j][2] = 0.0f;
          zc[j][0] = zc[j][1] = zc[j][2] = 0.0f;
          sig[j] = tau[j] = dist[j] = 0.0f;
        }
        lane_tau += tau[j];
        lane_sig += sig[j];
      }
      const float P = wave_excl_prefix(lane_tau, lane);
      float run = P;
      float lc[3] = {0.0f, 0.0f, 0.0f}, ld = 0.0f;
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        Sx[j] = run;
        const float T = expf(-run);
        const float alpha = -expm1f(-tau[j]);
        w[j] = valid ? T * alpha : 0.0f;
        run += tau[j];
        lc[0] = fmaf(w[j], c[j][0], lc[0]);
        lc[1] = fmaf(w[j], c[j][1], lc[1]);
        lc[2] = fmaf(w[j], c[j][2], lc[2]);
        ld = fmaf(w[j], dist[j], ld);
      }
      float Ch[3];
      Ch[0] = wave_sum(lc[0]);
      Ch[1] = wave_sum(lc[1]);
      Ch[2] = wave_sum(lc[2]);
      const float Dh = wave_sum(ld);
      const float Stot = wave_sum(lane_tau);
      const float Tend = expf(-Stot);

      if (mode == RM_MODE_FORWARD) {
        if (lane == 0) {
          if (a.out_rgb) {
            a.out_rgb[3 * ray] = Ch[0];
            a.out_rgb[3 * ray + 1] = Ch[1];
            a.out_rgb[3 * ray + 2] = Ch[2];
          }
          if (a.out_depth) a.out_depth[ray] = Dh;
          if (a.out_tend) a.out_tend[ray] = Tend;
        }
        continue;
      }

      float gC[3], gD = 0.0f, gT = 0.0f, dens = 0.0f;
      if (mode == RM_MODE_TRAIN) {
        // Eq. 7-11: squared colour error against the image (object rays) or
        // against the random colour with residual transmittance (background
        // rays), L1 depth term, density term on every background sample.
        float Co[3], l = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          Co[k] = bg ? fmaf(Tend, R.tgt[k], Ch[k]) : Ch[k];
          const float df = Co[k] - R.tgt[k];
          l = fmaf(df, df, l);
          gC[k] = 2.0f * df * invB;
        }
        if (!bg && (R.flags & RM_F_DEPTH)) {
          const float dd = Dh - R.D;
          l += a.lambda_depth * fabsf(dd);
          gD = a.lambda_depth * (dd > 0.0f ? 1.0f : (dd < 0.0f ? -1.0f : 0.0f)) * invB;
        }
        if (bg) {
          l += a.lambda_density * wave_sum(lane_sig);
          dens = a.lambda_density * invB;
        }
        loss_w += l * invB;
      } else {  // RM_MODE_ADJOINT
#pragma unroll
        for (int k = 0; k < 3; ++k) gC[k] = a.adj_rgb ? a.adj_rgb[3 * ray + k] : 0.0f;
        gD = a.adj_depth ? a.adj_depth[ray] : 0.0f;
        gT = a.adj_tend ? a.adj_tend[ray] : 0.0f;
      }
      // suffix sums  sum_{j > i} w_j c_j  and  sum_{j > i} w_j d_j
      const float Qc0 = wave_excl_suffix(lc[0], lane);
      const float Qc1 = wave_excl_suffix(lc[1], lane);
      const float Qc2 = wave_excl_suffix(lc[2], lane);
      const float Qd = wave_excl_suffix(ld, lane);
      float sc[3] = {Qc0, Qc1, Qc2}, sd = Qd;
      float bgterm = 0.0f;
      if (bg) bgterm = Tend * (gC[0] * R.tgt[0] + gC[1] * R.tgt[1] + gC[2] * R.tgt[2]);
#pragma unroll
      for (int j = SPL - 1; j >= 0; --j) {
        const int i = lane * SPL + j;
        const float Tn = expf(-(Sx[j] + tau[j]));
        float dtau = gC[0] * (Tn * c[j][0] - sc[0]) + gC[1] * (Tn * c[j][1] - sc[1]) +
                     gC[2] * (Tn * c[j][2] - sc[2]) + gD * (Tn * dist[j] - sd) - bgterm -
                     gT * Tend;
        const float dsig = dtau * R.delta + dens;
        sc[0] = fmaf(w[j], c[j][0], sc[0]);
        sc[1] = fmaf(w[j], c[j][1], sc[1]);
        sc[2] = fmaf(w[j], c[j][2], sc[2]);
        sd = fmaf(w[j], dist[j], sd);
        if (valid) {
          float* q = rv + i * 4;
          q[0] = y0[j] < 15.0f ? dsig * sig[j] : 0.0f;
#pragma unroll
          // sigmoid'(z) = sigmoid(z) sigmoid(-z): no cancellation where c rounds to 1
          for (int k = 0; k < 3; ++k) q[1 + k] = w[j] * gC[k] * c[j][k] * sigmoidf_(-zc[j][k]);
        }
      }
    }
    wave_lds_sync();

    // ---- backward: recompute activations per block, adjoints, dW ----
    if constexpr (PACKED) {
      // BF16, one hidden layer: blocks in pairs, so that each weight
      // gradient is one product over 32 samples (half the LDS round trips
      // and MFMA instructions of per-block products); activations recomputed
      // and rounded as in the forward, adjoints rounded once and used by
      // both their MFMA and their staging
#pragma unroll(KEEP_E ? NB / 2 : 1)
      for (int bp = 0; bp < NB; bp += 2) {
        bf16x4_t E2[2][KQ], H1b[2][4], Yb[2][1], H2b[2][4], dZb[2][1], dH2b[2][4], dYb[2][1],
            dH1b[2][4];
        float dy0[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int b = bp + h;
          if (KEEP_E) {
#pragma unroll
            for (int q = 0; q < KQ; ++q) E2[h][q] = EK[KEEP_E ? b : 0][q];
          } else {
            load_enc(sray + 16 * b + n, E2[h]);
          }
          floatx4 P[4], Yf[1];
          gemm_e(E2[h], P);
#pragma unroll
          for (int f = 0; f < 4; ++f) H1b[h][f] = relu_b(P[f]);
          MM::template gemm_b<16, 64>(wF2, H1b[h], Yf, lane);
          Yb[h][0] = cvt_bf16x4(Yf[0]);
          MM::template gemm_b<64, 16>(wF3, Yb[h], P, lane);
#pragma unroll
          for (int f = 0; f < 4; ++f) H2b[h][f] = relu_b(P[f]);
          floatx4 dz = {0.0f, 0.0f, 0.0f, 0.0f};
          dy0[h] = 0.0f;
          if (g == 0) {
            const float* q = rv + (16 * b + n) * 4;
            dy0[h] = q[0];
            dz = floatx4{q[1], q[2], q[3], 0.0f};
          }
          dZb[h][0] = cvt_bf16x4(dz);
        }
        // colour head: dW4 += dZ^T H2, dH2 = W4^T dZ masked by ReLU
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          MM::stage_b2(gbuf, dZb[h], 1, lane, 16 * h);
          MM::stage_b2(xbuf, H2b[h], 4, lane, 16 * h);
        }
        wave_lds_sync();
        MM::template dw32<16, 64>(gbuf, xbuf, acc4, lane);
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          floatx4 P[4];
          MM::template gemm_b<64, 16>(wB4, dZb[h], P, lane);
#pragma unroll
          for (int f = 0; f < 4; ++f) dH2b[h][f] = mask_b(P[f], H2b[h][f]);
        }
        // dW3 += dH2^T Y, dY = W3^T dH2 (+ density adjoint in row 0)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          MM::stage_b2(gbuf, dH2b[h], 4, lane, 16 * h);
          MM::stage_b2(xbuf, Yb[h], 1, lane, 16 * h);
        }
        wave_lds_sync();
        MM::template dw32<64, 16>(gbuf, xbuf, acc3, lane);
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          floatx4 dYf[1];
          MM::template gemm_b<16, 64>(wB3, dH2b[h], dYf, lane);
          if (g == 0) dYf[0][0] += dy0[h];
          dYb[h][0] = cvt_bf16x4(dYf[0]);
        }
        // dW2 += dY^T H1, dH1 = W2^T dY masked
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          MM::stage_b2(gbuf, dYb[h], 1, lane, 16 * h);
          MM::stage_b2(xbuf, H1b[h], 4, lane, 16 * h);
        }
        wave_lds_sync();
        MM::template dw32<16, 64>(gbuf, xbuf, acc2, lane);
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          floatx4 P[4];
          MM::template gemm_b<64, 16>(wB2, dYb[h], P, lane);
#pragma unroll
          for (int f = 0; f < 4; ++f) dH1b[h][f] = mask_b(P[f], H1b[h][f]);
        }
        // dW1 += dH1^T E, dE = W1^T dH1
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          MM::stage_b2(gbuf, dH1b[h], 4, lane, 16 * h);
          MM::stage_b2(xbuf, E2[h], KQ, lane, 16 * h);
        }
        wave_lds_sync();
        MM::template dw32<64, K1>(gbuf, xbuf, acc1, lane);
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          floatx4 dEf[KQ];
          MM::template gemm_b<K1, 64>(wB1, dH1b[h], dEf, lane);
          const int64_t s = sray + 16 * (bp + h) + n;
#pragma unroll
          for (int q = 0; q < KQ; ++q) {
            const int l0 = 8 * q + 2 * g, l1 = l0 + 1;
            if (l0 < L) a.de[(int64_t)l0 * S + s] = make_float2(dEf[q][0], dEf[q][1]);
            if (l1 < L) a.de[(int64_t)l1 * S + s] = make_float2(dEf[q][2], dEf[q][3]);
          }
        }
      }
      continue;
    }
#pragma unroll(KEEP_E ? NB : 1)
    for (int b = 0; b < NB; ++b) {
      const int64_t s = sray + 16 * b + n;
      etype E[KQ];
      floatx4 HH[NH][4], Y[1], H2[4];
      floatx4* H1 = HH[NH - 1];  // the last hidden layer of the density MLP
      if (KEEP_E) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) E[q] = EK[KEEP_E ? b : 0][q];
      } else {
        load_enc(s, E);
      }
      gemm_e(E, HH[0]);
      relu4(HH[0], 4);
#pragma unroll
      for (int k = 1; k < NH; ++k) {
        MM::template gemm<64, 64>(s_w + RM_OFF_HF(k), HH[k - 1], HH[k], lane);
        relu4(HH[k], 4);
      }
      MM::template gemm<16, 64>(wF2, H1, Y, lane);
      MM::template gemm<64, 16>(wF3, Y, H2, lane);
      relu4(H2, 4);
      floatx4 dZ[1], dH2[4], dY[1], dH1[4], dE[KQ];
      float dy0 = 0.0f;
      if (g == 0) {
        const float* q = rv + (16 * b + n) * 4;
        dy0 = q[0];
        dZ[0] = floatx4{q[1], q[2], q[3], 0.0f};
      } else {
        dZ[0] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
      }
      // colour head: dW4 += dZ^T H2, dH2 = W4^T dZ masked by ReLU
      MM::stage(gbuf, dZ, 1, lane);
      MM::stage(xbuf, H2, 4, lane);
      wave_lds_sync();
      MM::template dw<16, 64>(gbuf, xbuf, acc4, lane);
      wave_lds_sync();
      MM::template gemm<64, 16>(wB4, dZ, dH2, lane);
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) dH2[f][r] = H2[f][r] > 0.0f ? dH2[f][r] : 0.0f;
      // dW3 += dH2^T Y, dY = W3^T dH2 (+ density adjoint in row 0)
      MM::stage(gbuf, dH2, 4, lane);
      MM::stage(xbuf, Y, 1, lane);
      wave_lds_sync();
      MM::template dw<64, 16>(gbuf, xbuf, acc3, lane);
      wave_lds_sync();
      MM::template gemm<16, 64>(wB3, dH2, dY, lane);
      if (g == 0) dY[0][0] += dy0;
      // dW2 += dY^T H1, dH1 = W2^T dY masked
      MM::stage(gbuf, dY, 1, lane);
      MM::stage(xbuf, H1, 4, lane);
      wave_lds_sync();
      MM::template dw<16, 64>(gbuf, xbuf, acc2, lane);
      wave_lds_sync();
      MM::template gemm<64, 16>(wB2, dY, dH1, lane);
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) dH1[f][r] = H1[f][r] > 0.0f ? dH1[f][r] : 0.0f;
      // deeper density MLP, last layer first: dWh_k += dH^T H_{k-1},
      // dH <- Wh_k^T dH masked by ReLU
#pragma unroll
      for (int k = NH - 1; k >= 1; --k) {
        MM::stage(gbuf, dH1, 4, lane);
        MM::stage(xbuf, HH[k - 1], 4, lane);
        wave_lds_sync();
        MM::template dw<64, 64>(gbuf, xbuf, accH[k - 1], lane);
        wave_lds_sync();
        floatx4 dP[4];
        MM::template gemm<64, 64>(s_w + RM_OFF_HB(k), dH1, dP, lane);
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
          for (int r = 0; r < 4; ++r) dH1[f][r] = HH[k - 1][f][r] > 0.0f ? dP[f][r] : 0.0f;
      }
      // dW1 += dH^T E, dE = W1^T dH  (dH of the first hidden layer)
      MM::stage(gbuf, dH1, 4, lane);
      if constexpr (PREC == 1)
        MM::stage_b(xbuf, E, KQ, lane);
      else
        MM::stage(xbuf, E, KQ, lane);
      wave_lds_sync();
      MM::template dw<64, K1>(gbuf, xbuf, acc1, lane);
      wave_lds_sync();
      MM::template gemm<K1, 64>(wB1, dH1, dE, lane);
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const int l0 = 8 * q + 2 * g, l1 = l0 + 1;
        if (l0 < L) a.de[(int64_t)l0 * S + s] = make_float2(dE[q][0], dE[q][1]);
        if (l1 < L) a.de[(int64_t)l1 * S + s] = make_float2(dE[q][2], dE[q][3]);
      }
    }
  }

  // ---- work-item record: weight gradients in parameter order, and loss ----
  // The waves' partial sums are combined in turn (wave 0 stores, waves 1..3
  // add), with plain LDS accesses: each wave covers every record entry once,
  // and float atomics in LDS are slow.  The order is fixed, so the record is
  // deterministic.
  if (mode != RM_MODE_FORWARD) {
    const int oh = RM_HIDDEN * din, o2 = oh + (NH - 1) * RM_HH, o3 = o2 + RM_DOUT * RM_HIDDEN,
              o4 = o3 + RM_HIDDEN * RM_GEO;
    if (ALIAS) __syncthreads();  // the record overwrites the weights: every wave is done
    for (int turn = 0; turn < RM_WG / 64; ++turn) {
      if (wave == turn) {
        const bool first = turn == 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 4 * g + r;
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < KQ; ++u) {
              const int m = 16 * t + row, k = 16 * u + n;
              if (k < din) {
                float* d = &s_rec[m * din + k];
                *d = first ? acc1[t * KQ + u][r] : *d + acc1[t * KQ + u][r];
              }
            }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            float* d = &s_rec[o2 + row * RM_HIDDEN + 16 * u + n];
            *d = first ? acc2[u][r] : *d + acc2[u][r];
          }
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (n >= 1) {
              float* d = &s_rec[o3 + (16 * t + row) * RM_GEO + (n - 1)];
              *d = first ? acc3[t][r] : *d + acc3[t][r];
            }
          if (row < 3)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              float* d = &s_rec[o4 + row * RM_HIDDEN + 16 * u + n];
              *d = first ? acc4[u][r] : *d + acc4[u][r];
            }
#pragma unroll
          for (int k = 0; k < NH - 1; ++k)
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                float* d = &s_rec[oh + k * RM_HH + (16 * tt + row) * RM_HIDDEN + 16 * u + n];
                *d = first ? accH[k][tt * 4 + u][r] : *d + accH[k][tt * 4 + u][r];
              }
        }
        if (lane == 0) s_rec[RL] = first ? loss_w : s_rec[RL] + loss_w;
      }
      __syncthreads();
    }
    float* rec = a.partials + (int64_t)blockIdx.x * RM_REC_STRIDE_NH(NH);
    for (int j = tid; j < RL + 1; j += RM_WG) rec[j] = s_rec[j];
  }
}

// ---------------------------------------------------------------------------
// K5: per-object MLP gradient and loss from the work-item records, summed in
// a fixed order (deterministic); in a training step the MLP's Adam update is
// applied here, else the gradient is written.  A block owns
// 256 record columns, 4 per lane (column RM_REC_LOSS_NH is the loss); its 16
// waves sum interleaved sixteenths of the items, then combine in LDS.
__global__ __launch_bounds__(RM_RED_WG) void k_reduce(StepArgs a) {
  constexpr int NW = RM_RED_WG / 64;
  __shared__ float4 s_part[NW][64];
  const StepObj so = a.sobj[blockIdx.y];
  const ObjStatic& ob = a.objs[so.obj];
  const int nm = (int)(ob.P - ob.P_grid);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = blockIdx.x * 256 + 4 * lane;  // 4 columns per lane (the stride is a multiple of 4)
  float4 s[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) s[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const int stride = RM_REC_STRIDE_NH(a.mlp_layers), rloss = RM_REC_LOSS_NH(a.mlp_layers);
  if (j0 < stride) {
    // wave w sums items w, w + NW, ...: four per lane in flight, each into
    // its own partial sum (a fixed order: deterministic)
    const float* col = a.partials + j0;
    for (int it = so.item_begin + wave; it < so.item_end; it += 4 * NW) {
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        x[u] = it + u * NW < so.item_end ? *(const float4*)(col + (int64_t)(it + u * NW) * stride)
                                         : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s[u].x += x[u].x; s[u].y += x[u].y; s[u].z += x[u].z; s[u].w += x[u].w;
      }
    }
  }
  s_part[wave][lane] = make_float4((s[0].x + s[1].x) + (s[2].x + s[3].x),
                                   (s[0].y + s[1].y) + (s[2].y + s[3].y),
                                   (s[0].z + s[1].z) + (s[2].z + s[3].z),
                                   (s[0].w + s[1].w) + (s[2].w + s[3].w));
  __syncthreads();
  if (wave != 0 || j0 >= stride) return;
  float4 t = s_part[0][lane];
#pragma unroll
  for (int w = 1; w < NW; ++w) {  // fixed order: deterministic
    const float4 u = s_part[w][lane];
    t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
  }
  const float tv[4] = {t.x, t.y, t.z, t.w};
  float* gdst = a.grad_override ? a.grad_override : ob.grad;
  const float bc1 = a.state[so.obj].bc1, bc2 = a.state[so.obj].bc2;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = j0 + c;
    if (j < nm) {
      const int64_t o = ob.P_grid + j;
      if (a.fuse_adam) {  // training step: the MLP gradient is complete here
        adam1(ob.params[o], ob.m[o], ob.v[o], tv[c], a, bc1, bc2);
      } else {
        gdst[o] = tv[c];
      }
    } else if (j == rloss && a.mode == RM_MODE_TRAIN) {
      ObjState* st = a.state + so.obj;
      st->loss_acc += tv[c];
      st->n_loss += 1;
    }
  }
}


// ---------------------------------------------------------------------------
// Density of an object's field at a normalised position p in [0,1]^3:
// encoding + density head on VALU.  DEEP: the density MLP has hidden-to-hidden
// layers (compiled apart, so the one-layer kernels keep their registers).
template <bool DEEP>
__device__ inline float density_p(const ObjStatic& ob, const float p[3]) {
  // loops over the largest level count with guards: constant indices keep
  // the encoding in registers
  float e[2 * RM_MAX_LEVELS];
#pragma unroll
  for (int l = 0; l < RM_MAX_LEVELS; ++l) {
    float ex = 0.0f, ey = 0.0f;
    if (l < ob.L) {
      Cell cl;
      make_cell(p, ob.N_l[l], cl);
      const bool hashed = (ob.hashed_mask >> l) & 1u;
      const float* G = ob.params + ob.off[l];
      for (int b = 0; b < 8; ++b) {
        const uint32_t id = corner_index(cl, b, ob.N_l[l], ob.T_l[l], hashed);
        const float w = corner_weight(cl, b);
        ex = fmaf(w, G[2 * (int64_t)id], ex);
        ey = fmaf(w, G[2 * (int64_t)id + 1], ey);
      }
    }
    e[2 * l] = ex;
    e[2 * l + 1] = ey;
  }
  const float* W1 = ob.params + ob.P_grid;
  const float* Wh = W1 + RM_HIDDEN * ob.din;
  const float* W2 = Wh + (ob.mlp_layers - 1) * RM_HH;
  float y0 = 0.0f;
  if (!DEEP) {
    for (int h = 0; h < RM_HIDDEN; ++h) {
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < 2 * RM_MAX_LEVELS; ++k)
        if (k < ob.din) s = fmaf(W1[h * ob.din + k], e[k], s);
      y0 = fmaf(W2[h], s > 0.0f ? s : 0.0f, y0);
    }
  } else {
    float ha[RM_HIDDEN], hb[RM_HIDDEN];
    for (int h = 0; h < RM_HIDDEN; ++h) {
      float s = 0.0f;
      for (int k = 0; k < ob.din; ++k) s = fmaf(W1[h * ob.din + k], e[k], s);
      ha[h] = s > 0.0f ? s : 0.0f;
    }
    for (int k = 1; k < ob.mlp_layers; ++k) {
      const float* H = Wh + (k - 1) * RM_HH;
      for (int h = 0; h < RM_HIDDEN; ++h) {
        float s = 0.0f;
        for (int j = 0; j < RM_HIDDEN; ++j) s = fmaf(H[h * RM_HIDDEN + j], ha[j], s);
        hb[h] = s > 0.0f ? s : 0.0f;
      }
      for (int h = 0; h < RM_HIDDEN; ++h) ha[h] = hb[h];
    }
    for (int h = 0; h < RM_HIDDEN; ++h) y0 = fmaf(W2[h], ha[h], y0);
  }
  return expf(fminf(y0, 15.0f));
}

// density at an object-frame point (meshing, queries)
template <bool DEEP>
__device__ inline float density_at(const ObjStatic& ob, const float x[3]) {
  float p[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float q = (x[k] + ob.half[k]) / (ob.half[k] + ob.half[k]);
    p[k] = fminf(fmaxf(q, 0.0f), 1.0f);
  }
  return density_p<DEEP>(ob, p);
}

template <bool DEEP>
__global__ __launch_bounds__(256) void k_query_density(const ObjStatic* objs, int obj,
                                                       const float* xyz, int64_t n, float* sigma) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float x[3] = {xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2]};
  sigma[t] = density_at<DEEP>(objs[obj], x);
}

// ---------------------------------------------------------------------------
// Meshing: marching cubes (Lorensen & Cline) over a (res+1)^3 corner grid,
// x fastest, corner (i, j, k) at lo + (hi - lo) * (i, j, k) / res.

__device__ inline float grid_coord(float lo, float hi, int g, int res) {
  return lo + (hi - lo) * ((float)g / (float)res);
}

// density of an object at the corners of a grid over its box
template <bool DEEP>
__global__ __launch_bounds__(256) void k_density_grid(const ObjStatic* objs, int obj, int res,
                                                      float* grid) {
  const int64_t n1 = res + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n1 * n1 * n1) return;
  const ObjStatic& ob = objs[obj];
  const int g[3] = {(int)(t % n1), (int)((t / n1) % n1), (int)(t / (n1 * n1))};
  float x[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = grid_coord(-ob.half[a], ob.half[a], g[a], res);
  grid[t] = density_at<DEEP>(ob, x);
}

// case of cell c and its 8 corner values
__device__ inline int mc_cell(const MeshArgs& m, int64_t c, float v[8], int g0[3]) {
  const int64_t n1 = m.res + 1;
  g0[0] = (int)(c % m.res);
  g0[1] = (int)((c / m.res) % m.res);
  g0[2] = (int)(c / ((int64_t)m.res * m.res));
  int mask = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int64_t gi = (g0[0] + (k & 1)) + n1 * ((g0[1] + ((k >> 1) & 1)) + n1 * (g0[2] + (k >> 2)));
    v[k] = m.grid[gi];
    mask |= (v[k] > m.iso ? 1 : 0) << k;
  }
  return mask;
}

__global__ __launch_bounds__(256) void k_mc_count(MeshArgs m) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)m.res * m.res * m.res) return;
  float v[8];
  int g0[3];
  m.cnt[c] = m.ntri[mc_cell(m, c, v, g0)];
}

// exclusive scan of cnt[0 .. n) in blocks of RM_MC_SCAN (in place); block totals to bsum
__global__ __launch_bounds__(256) void k_mc_scan_blocks(int* cnt, int64_t n, int* bsum) {
  __shared__ int s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * RM_MC_SCAN + 4 * tid;  // 4 consecutive per thread
  int x[4], mine = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = b0 + k < n ? cnt[b0 + k] : 0;
    mine += x[k];
  }
  int inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wave; ++w) off += s_w[w];
  int run = off + inc - mine;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (b0 + k < n) cnt[b0 + k] = run;
    run += x[k];
  }
  if (tid == 255) bsum[blockIdx.x] = off + inc;
}

// exclusive scan of the block totals (nb <= 4 * 1024) in one block; total to bsum[nb]
__global__ __launch_bounds__(1024) void k_mc_scan_totals(int* bsum, int nb) {
  __shared__ int s_w[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int x[4], mine = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = 4 * tid + k < nb ? bsum[4 * tid + k] : 0;
    mine += x[k];
  }
  int inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) off += s_w[w];
    tot += s_w[w];
  }
  int run = off + inc - mine;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (4 * tid + k < nb) bsum[4 * tid + k] = run;
    run += x[k];
  }
  if (tid == 0) bsum[nb] = tot;
}

__global__ __launch_bounds__(256) void k_mc_emit(MeshArgs m) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)m.res * m.res * m.res) return;
  float v[8];
  int g0[3];
  const int mask = mc_cell(m, c, v, g0);
  const int nt = m.ntri[mask];
  if (nt == 0) return;
  const int64_t base = (int64_t)m.cnt[c] + m.bsum[c / RM_MC_SCAN];
  for (int t = 0; t < nt; ++t) {
    if (base + t >= m.max_tris) return;
    float* o = m.out + 9 * (base + t);
    for (int q = 0; q < 3; ++q) {
      const int e = m.tris[16 * mask + 3 * t + q];
      const int ca = m.edge_a[e], cb = m.edge_b[e];
      const float s = (m.iso - v[ca]) / (v[cb] - v[ca]);
      float x[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float xa = grid_coord(m.lo[a], m.hi[a], g0[a] + ((ca >> a) & 1), m.res);
        const float xb = grid_coord(m.lo[a], m.hi[a], g0[a] + ((cb >> a) & 1), m.res);
        x[a] = xa + s * (xb - xa);
      }
      if (m.world) {  // box pose: x_w = R x + t
#pragma unroll
        for (int a = 0; a < 3; ++a)
          o[3 * q + a] = ((m.R[3 * a] * x[0] + m.R[3 * a + 1] * x[1]) + m.R[3 * a + 2] * x[2]) + m.t[a];
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) o[3 * q + a] = x[a];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_debug_encode(const ObjStatic* objs, int obj,
                                                      const float* pts, int64_t n, uint32_t* idx,
                                                      float* feat) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const ObjStatic& ob = objs[obj];
  const float p[3] = {pts[3 * t], pts[3 * t + 1], pts[3 * t + 2]};
  for (int l = 0; l < ob.L; ++l) {
    Cell cl;
    make_cell(p, ob.N_l[l], cl);
    const bool hashed = (ob.hashed_mask >> l) & 1u;
    const float* G = ob.params + ob.off[l];
    float ex = 0.0f, ey = 0.0f;
    for (int b = 0; b < 8; ++b) {
      const uint32_t id = corner_index(cl, b, ob.N_l[l], ob.T_l[l], hashed);
      const float w = corner_weight(cl, b);
      if (idx) idx[(t * ob.L + l) * 8 + b] = id;
      ex = fmaf(w, G[2 * (int64_t)id], ex);
      ey = fmaf(w, G[2 * (int64_t)id + 1], ey);
    }
    if (feat) {
      feat[(t * ob.L + l) * 2] = ex;
      feat[(t * ob.L + l) * 2 + 1] = ey;
    }
  }
}

// parameter initialisation: grid U(-1e-4, 1e-4), MLP Glorot-uniform, each
// value drawn from Philox with counter (index, kind, 0xFFFFFFFF, 0)
__global__ __launch_bounds__(256) void k_init_params(float* params, int64_t P_grid, int din,
                                                     int nh, uint32_t k0, uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n1 = (int64_t)RM_HIDDEN * din, nhh = n1 + (int64_t)(nh - 1) * RM_HH;
  const int64_t n2 = nhh + RM_DOUT * RM_HIDDEN;
  const int64_t n3 = n2 + RM_HIDDEN * RM_GEO, n4 = n3 + 3 * RM_HIDDEN;
  if (i >= P_grid + n4) return;
  uint32_t kind;
  float lim;
  if (i < P_grid) {
    kind = 0u;
    lim = 1e-4f;
  } else {
    const int64_t j = i - P_grid;
    if (j < n1) { kind = 1u; lim = sqrtf(6.0f / (float)(RM_HIDDEN + din)); }
    else if (j < nhh) { kind = 5u; lim = sqrtf(6.0f / (float)(2 * RM_HIDDEN)); }
    else if (j < n2) { kind = 2u; lim = sqrtf(6.0f / (float)(RM_DOUT + RM_HIDDEN)); }
    else if (j < n3) { kind = 3u; lim = sqrtf(6.0f / (float)(RM_HIDDEN + RM_GEO)); }
    else { kind = 4u; lim = sqrtf(6.0f / (float)(3 + RM_HIDDEN)); }
  }
  uint32_t x[4];
  philox4x32_10((uint32_t)i, kind, 0xFFFFFFFFu, 0u, k0, k1, x);
  const float u = (float)(x[0] >> 8) * (1.0f / 16777216.0f);
  params[i] = (2.0f * u - 1.0f) * lim;
}

// sample positions of a launch's rays (inspection)
template <int NS>
__global__ __launch_bounds__(256) void k_debug_positions(StepArgs a, float* pos) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.S) return;
  const RayRec R = a.rays[s / NS];
  float p[3] = {0.0f, 0.0f, 0.0f};
  if (R.flags & RM_F_HIT) sample_pos(R, (int)(s % NS), a.objs[R.obj].half, p);
  pos[3 * s] = p[0];
  pos[3 * s + 1] = p[1];
  pos[3 * s + 2] = p[2];
}

// clears the per-object loss accumulators of a launch's objects
__global__ void k_reset_loss(StepArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_sobj) return;
  ObjState* st = a.state + a.sobj[i].obj;
  st->loss_acc = 0.0f;
  st->n_loss = 0;
}

// occupancy refresh: bit = density at the cell centre > threshold; a wave
// covers 64 consecutive cells and stores its two words from a ballot
template <bool DEEP>
__global__ __launch_bounds__(256) void k_occ_update(const ObjStatic* objs, int obj,
                                                   uint32_t* bits, float threshold) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;  // < 64^3, grid exact
  const ObjStatic& ob = objs[obj];
  const float p[3] = {((float)(cell & 63) + 0.5f) / 64.0f,
                      ((float)((cell >> 6) & 63) + 0.5f) / 64.0f,
                      ((float)(cell >> 12) + 0.5f) / 64.0f};
  const bool on = density_p<DEEP>(ob, p) > threshold;
  const uint64_t m = __ballot(on);
  const int lane = threadIdx.x & 63;
  if (lane < 2) bits[(cell >> 5) + lane] = (uint32_t)(m >> (32 * lane));
}

__global__ void k_fill(float* x, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ---------------------------------------------------------------------------
// launchers

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

#define RM_NS_SWITCH(NS, CALL)              \
  switch (NS) {                             \
    case 32: { constexpr int NSC = 32; CALL; break; }   \
    case 64: { constexpr int NSC = 64; CALL; break; }   \
    case 128: { constexpr int NSC = 128; CALL; break; } \
    default: return hipErrorInvalidValue;   \
  }

hipError_t rm_launch_raygen(const StepArgs& a, int NS, hipStream_t st) {
  if (a.n_rays <= 0) return hipSuccess;
  RM_NS_SWITCH(NS, (k_raygen<NSC><<<cdiv(a.n_rays, 256), 256, 0, st>>>(a)));
  return hipGetLastError();
}

hipError_t rm_launch_encode_fwd(const StepArgs& a, int NS, int block, hipStream_t st) {
  if (a.n_bblocks <= 0) return hipSuccess;
  const int nwg = a.n_bblocks * RM_ENC_SPLIT;  // rounded up to whole rounds of the 8 XCDs
  RM_NS_SWITCH(NS, (k_encode_fwd<NSC><<<8 * ((nwg + 7) / 8), block, 0, st>>>(a)));
  return hipGetLastError();
}

hipError_t rm_launch_bin_scatter(const StepArgs& a, const BinGroup& g, int NS, hipStream_t st) {
  if (g.bb_end <= g.bb_begin) return hipSuccess;
  const size_t lds = (size_t)RM_SCAT_WG * 8 * 12 + (size_t)a.bin_max_R * 3 * sizeof(int);
  if (lds > 65536) {  // beyond the default dynamic LDS limit (tables of 2^22+ entries)
    hipError_t e0 = hipSuccess;
    RM_NS_SWITCH(NS, (e0 = hipFuncSetAttribute((const void*)k_bin_scatter<NSC>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds)));
    if (e0 != hipSuccess) return e0;
  }
  StepArgs b = a;
  b.bb_begin = g.bb_begin;
  b.n_bblocks = g.bb_end - g.bb_begin;  // the group's blocks
  RM_NS_SWITCH(NS, (k_bin_scatter<NSC><<<8 * ((b.n_bblocks + 7) / 8), RM_SCAT_WG, lds, st>>>(b)));
  return hipGetLastError();
}

hipError_t rm_launch_bin_acc(const StepArgs& a, const BinGroup& g, hipStream_t st) {
  if (g.bin_end <= g.bin_begin) return hipSuccess;
  StepArgs b = a;
  b.bin_begin = g.bin_begin;
  k_bin_acc<<<g.bin_end - g.bin_begin, RM_ACC_WG, 0, st>>>(b);
  return hipGetLastError();
}

hipError_t rm_launch_pack(const StepArgs& a, int K1, hipStream_t st) {
  if (a.n_sobj <= 0) return hipSuccess;
  if (a.mlp_layers < 1 || a.mlp_layers > RM_MAX_MLP_LAYERS) return hipErrorInvalidValue;
  k_pack<<<dim3(a.n_sobj, 8 + 2 * (a.mlp_layers - 1)), 256, 0, st>>>(a, K1);
  return hipGetLastError();
}

template <int PREC, int K1, int NH>
static hipError_t launch_field_k(const StepArgs& a, int NS, hipStream_t st) {
  RM_NS_SWITCH(NS, (k_field<PREC, NSC, K1, NH><<<a.n_items, RM_WG, 0, st>>>(a)));
  return hipGetLastError();
}

template <int NH>
static hipError_t launch_field_nh(const StepArgs& a, int NS, int K1, int prec, hipStream_t st) {
  if (K1 == 16)
    return prec ? launch_field_k<1, 16, NH>(a, NS, st) : launch_field_k<0, 16, NH>(a, NS, st);
  if (K1 == 32)
    return prec ? launch_field_k<1, 32, NH>(a, NS, st) : launch_field_k<0, 32, NH>(a, NS, st);
  return hipErrorInvalidValue;
}

hipError_t rm_launch_field(const StepArgs& a, int NS, int K1, int prec, hipStream_t st) {
  if (a.n_items <= 0) return hipSuccess;
  switch (a.mlp_layers) {
    case 1: return launch_field_nh<1>(a, NS, K1, prec, st);
    case 2: return launch_field_nh<2>(a, NS, K1, prec, st);
    case 3: return launch_field_nh<3>(a, NS, K1, prec, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t rm_launch_reduce(const StepArgs& a, hipStream_t st) {
  if (a.n_sobj <= 0) return hipSuccess;
  dim3 grid(cdiv(RM_REC_LOSS_NH(a.mlp_layers) + 1, 256), a.n_sobj);
  k_reduce<<<grid, RM_RED_WG, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t rm_launch_bin_finish(const StepArgs& a, hipStream_t st) {
  if (a.n_fins <= 0 || !a.fuse_adam) return hipSuccess;
  k_bin_finish<<<a.n_fins, RM_FIN_WG, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t rm_launch_camera_rays(const StepArgs& a, int NS, const float* M, const float* c,
                                 float fx, float fy, float cx, float cy, int W, int pix0,
                                 hipStream_t st) {
  if (a.n_rays <= 0) return hipSuccess;
  CamArgs ca;
  for (int k = 0; k < 9; ++k) ca.M[k] = M[k];
  for (int k = 0; k < 3; ++k) ca.c[k] = c[k];
  ca.fx = fx;
  ca.fy = fy;
  ca.cx = cx;
  ca.cy = cy;
  ca.W = W;
  ca.pix0 = pix0;
  RM_NS_SWITCH(NS, (k_camera_rays<NSC><<<cdiv(a.n_rays, 256), 256, 0, st>>>(a, ca)));
  return hipGetLastError();
}

hipError_t rm_launch_user_rays(const StepArgs& a, int NS, const float* rays, hipStream_t st) {
  if (a.n_rays <= 0) return hipSuccess;
  RM_NS_SWITCH(NS, (k_user_rays<NSC><<<cdiv(a.n_rays, 256), 256, 0, st>>>(a, rays)));
  return hipGetLastError();
}

hipError_t rm_launch_query_density(const ObjStatic* objs, int obj, int nh, const float* xyz,
                                   int64_t n, float* sigma, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (nh > 1) k_query_density<true><<<cdiv(n, 256), 256, 0, st>>>(objs, obj, xyz, n, sigma);
  else k_query_density<false><<<cdiv(n, 256), 256, 0, st>>>(objs, obj, xyz, n, sigma);
  return hipGetLastError();
}

hipError_t rm_launch_density_grid(const ObjStatic* objs, int obj, int nh, int res, float* grid,
                                  hipStream_t st) {
  const int64_t n1 = res + 1;
  if (nh > 1) k_density_grid<true><<<cdiv(n1 * n1 * n1, 256), 256, 0, st>>>(objs, obj, res, grid);
  else k_density_grid<false><<<cdiv(n1 * n1 * n1, 256), 256, 0, st>>>(objs, obj, res, grid);
  return hipGetLastError();
}

hipError_t rm_launch_mc_count(const MeshArgs& m, hipStream_t st) {
  const int64_t nc = (int64_t)m.res * m.res * m.res;
  k_mc_count<<<cdiv(nc, 256), 256, 0, st>>>(m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = (int)cdiv(nc, RM_MC_SCAN);
  k_mc_scan_blocks<<<nb, 256, 0, st>>>(m.cnt, nc, m.bsum);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_mc_scan_totals<<<1, 1024, 0, st>>>(m.bsum, nb);
  return hipGetLastError();
}

hipError_t rm_launch_mc_emit(const MeshArgs& m, hipStream_t st) {
  const int64_t nc = (int64_t)m.res * m.res * m.res;
  k_mc_emit<<<cdiv(nc, 256), 256, 0, st>>>(m);
  return hipGetLastError();
}

hipError_t rm_launch_debug_encode(const ObjStatic* objs, int obj, const float* p, int64_t n,
                                  uint32_t* idx, float* feat, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_debug_encode<<<cdiv(n, 256), 256, 0, st>>>(objs, obj, p, n, idx, feat);
  return hipGetLastError();
}

hipError_t rm_launch_init(float* params, int64_t P_grid, int din, int nh, uint32_t k0,
                          uint32_t k1, hipStream_t st) {
  const int64_t n = P_grid + (int64_t)RM_HIDDEN * din + (int64_t)(nh - 1) * RM_HH +
                    RM_DOUT * RM_HIDDEN + RM_HIDDEN * RM_GEO + 3 * RM_HIDDEN;
  k_init_params<<<cdiv(n, 256), 256, 0, st>>>(params, P_grid, din, nh, k0, k1);
  return hipGetLastError();
}

hipError_t rm_launch_debug_positions(const StepArgs& a, int NS, float* pos, hipStream_t st) {
  if (a.S <= 0) return hipSuccess;
  RM_NS_SWITCH(NS, (k_debug_positions<NSC><<<cdiv(a.S, 256), 256, 0, st>>>(a, pos)));
  return hipGetLastError();
}

hipError_t rm_launch_reset_loss(const StepArgs& a, hipStream_t st) {
  if (a.n_sobj <= 0) return hipSuccess;
  k_reset_loss<<<cdiv(a.n_sobj, 64), 64, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t rm_launch_occ_update(const ObjStatic* objs, int obj, int nh, uint32_t* bits,
                                float threshold, hipStream_t st) {
  if (nh > 1) k_occ_update<true><<<(64 * 64 * 64) / 256, 256, 0, st>>>(objs, obj, bits, threshold);
  else k_occ_update<false><<<(64 * 64 * 64) / 256, 256, 0, st>>>(objs, obj, bits, threshold);
  return hipGetLastError();
}

hipError_t rm_launch_fill(float* x, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill<<<cdiv(n, 256), 256, 0, st>>>(x, n, v);
  return hipGetLastError();
}
