// romap_device.h -- data layouts shared by the gfx950 kernels and the host
// runtime of libromap.  Internal to the library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RM_MAX_LEVELS 16
#define RM_HIDDEN 64
#define RM_GEO 15
#define RM_DOUT 16
#define RM_MLP_MAX (64 * 32 + 16 * 64 + 64 * 15 + 3 * 64) /* 4224 */
#define RM_WPACK 10240      /* packed MLP weight image, elements (K1 <= 32) */
#define RM_MAX_MLP_LAYERS 3 /* hidden layers of the density MLP: 1 (Sec. V), 2, 3 (Table 4) */
// with nh hidden layers: nh - 1 more 64 x 64 matrices in the parameters,
// their gradients in the work-item records and two operand images each
#define RM_HH (RM_HIDDEN * RM_HIDDEN)
#define RM_MLP_NH(nh) (RM_MLP_MAX + ((nh) - 1) * RM_HH)      /* MLP floats, K1 = 32 */
#define RM_REC_LOSS_NH(nh) RM_MLP_NH(nh)   /* work-item record: MLP gradients, then the loss */
#define RM_REC_STRIDE_NH(nh) (RM_REC_LOSS_NH(nh) + 16)  /* floats per record, padded */
#define RM_WPACK_NH(nh) (RM_WPACK + ((nh) - 1) * 2 * RM_HH)
#define RM_OFF_HF(k) (RM_WPACK + ((k) - 1) * 2 * RM_HH)     /* Wh_k   64 x 64 */
#define RM_OFF_HB(k) (RM_OFF_HF(k) + RM_HH)                 /* Wh_k^T 64 x 64 */
#define RM_WG 256           /* threads of the fused field kernel (4 waves) */
#define RM_FIN_WG 512       /* entries per workgroup of the finishing kernel */
// Threads of the MLP reduction: small workgroups start beside the other
// object group's kernels as soon as one of theirs finishes (with 1024 the
// kernel took 86-144 us there against 11 us alone; with 256, 34-43 us; step
// 1.710 -> 1.702 ms on 24 objects, 512: 1.703).
#ifndef RM_RED_WG
#define RM_RED_WG 256
#endif
#define RM_GRAPH_MIN_STEPS 8 /* steps of a romap_train call that repay a graph capture */
#ifndef RM_GRAPH_STEPS
#define RM_GRAPH_STEPS 4     /* training steps captured in one graph */
#endif
// Work share of the first group of a two-stream step (the second starts
// once the first has passed its gather); measured on 24 objects, ms per
// step (two runs each): 0.4 1.718, 0.45 1.722 1.719, 0.5 1.705 1.703,
// 0.55 1.709 1.705, 0.6 1.756.
#ifndef RM_SPLIT_SHARE
#define RM_SPLIT_SHARE 0.50
#endif
// The binning merges the corners consecutive samples of a ray share on
// levels with N_l <= NUM/DEN * samples per ray (NUM/DEN = 2, 4, 8: 1.741,
// 1.742, 1.746 ms per step on 24 objects; finer levels rarely share any).
#ifndef RM_MERGE_NUM
#define RM_MERGE_NUM 4
#define RM_MERGE_DEN 1
#endif
#define RM_RB_BITS 11       /* binned scatter: table entries per region = 2048 */
#define RM_RB (1 << RM_RB_BITS)
#define RM_ACC_WG 512       /* threads of the region accumulation kernel */
#ifndef RM_SCAT_WG
#define RM_SCAT_WG 512      /* samples (threads) per block of the binning kernel */
#endif
#ifndef RM_ENC_SPLIT
#define RM_ENC_SPLIT 2      /* gather workgroups per block (measured: 1, 2, 4 -> 535, 512, 517 us) */
#endif
#define RM_ACC_CHUNK 32768  /* records per accumulation workgroup (about; 8192, 16384, 32768: 2.33, 2.23, 2.22 ms per step) */
#define RM_ACC_MAXK 256     /* accumulation workgroups per region, at most */
#ifndef RM_GROUP_RECORDS
#define RM_GROUP_RECORDS (1ll << 29) /* record slots of one bin group (4 GiB) */
#endif
#ifndef RM_ACC_RQ
#define RM_ACC_RQ 4         /* quads of records per thread the accumulation keeps in registers */
#endif
#define RM_FX_BITS 38       /* fixed-point fraction bits of the region sums */
#define RM_MAX_REGIONS 8192 /* 2^24 / 2^11 */

// Offsets of the eight packed GEMM operands inside a weight image.
#define RM_OFF_F1 0     /* W1        64 x K1  */
#define RM_OFF_F2 2048  /* W2        16 x 64  */
#define RM_OFF_F3 3072  /* W3'       64 x 16  (column 0 = 0, k>=1 -> W3[.][k-1]) */
#define RM_OFF_F4 4096  /* W4 padded 16 x 64  */
#define RM_OFF_B4 5120  /* W4'^T     64 x 16  */
#define RM_OFF_B3 6144  /* W3'^T     16 x 64  */
#define RM_OFF_B2 7168  /* W2^T      64 x 16  */
#define RM_OFF_B1 8192  /* W1^T      K1 x 64  */

// ray classes (Sec. V-B) and flags
#define RM_CLS_OCCLUDER 0
#define RM_CLS_OBJECT 1
#define RM_CLS_BACKGROUND 2
#define RM_F_CLS 3u
#define RM_F_HIT 4u
#define RM_F_DEPTH 8u

// kernel modes of the fused field kernel
#define RM_MODE_TRAIN 0   /* loss of Eq. 7-11 against the ray targets, then adjoint */
#define RM_MODE_FORWARD 1 /* colour, depth, T_end only */
#define RM_MODE_ADJOINT 2 /* adjoint of caller-given output gradients */

struct KfRef {          // one accepted keyframe of one object
  int32_t kf;           // global keyframe slot
  int32_t x0, y0, w, h; // candidate rectangle
  float M[9];           // camera -> object rotation
  float c[3];           // camera centre in the object frame
  int32_t pad;
  int64_t cand_begin;   // candidates of the object's earlier keyframes
};

struct KfDev {
  const uint8_t* rgb;
  const int32_t* mask;
  const float* depth;   // may be null
  int32_t W, H;
  float fx, fy, cx, cy;
};

struct ObjStatic {      // written by the host
  float* params;        // P_alloc floats: grid (P_grid) then MLP
  float* grad;
  float* m;
  float* v;
  int64_t P, P_grid, P_alloc;
  int64_t off[RM_MAX_LEVELS + 1]; // level offsets in floats
  uint32_t N_l[RM_MAX_LEVELS];
  uint32_t T_l[RM_MAX_LEVELS];
  uint32_t hashed_mask;
  int32_t L, din, instance, id, n_kf;
  float half[3];
  int32_t mlp_layers;   // hidden layers of the density MLP
  const KfRef* kfs;
  int64_t n_cand;
  const uint32_t* occ;  // 64^3 occupancy bits, or null (no skipping)
};

struct ObjState {       // written by the device
  int32_t step;         // Adam steps taken
  float bc1, bc2;       // 1 - beta^step of the current step
  float loss_acc;       // sum of per-step losses since the host last read it
  int32_t n_loss;
  int32_t pad[3];
};

struct RayRec {         // 64 B
  float o[3], d[3];
  float tn, delta;
  float tgt[3];         // image colour (object rays) or random colour (background)
  float D;              // depth target (ray distance)
  uint32_t flags;
  int32_t obj;
  int32_t pad0, pad1;
};

struct StepObj {        // one object of a launch
  int32_t obj;
  int32_t n_rays;       // B_o, the loss normaliser
  int32_t ray_begin;
  int32_t item_begin, item_end;
  int32_t pad[3];
};

struct Item {           // one workgroup of the fused field kernel
  int32_t so;
  int32_t ray_begin;
  int32_t n_rays;
  int32_t pad;
};

struct Fin {            // one workgroup of the finishing kernel: RM_FIN_WG
  int32_t pair, region; // entries of a region that several workgroups summed
  int32_t sub, pad;
};

struct BinPair {        // one (object of the launch, binned level)
  int32_t so, l;
  int32_t nb;           // sample blocks of RM_SCAT_WG of the object
  int32_t R;            // regions of the level's table
  int64_t rec_base;     // first record slot of this pair
  int32_t bin_base;     // first bin (region) of this pair
  int32_t cap;          // record slots per bin (multiple of 4)
  int32_t K;            // accumulation workgroups per bin
  int32_t merge;        // coarse dense level: merge runs of samples in one cell
  int64_t s_begin;      // first sample of the object
  int64_t n_samples;
};

struct BinBlock {       // one block of RM_SCAT_WG samples of one binned pair
  int32_t pair, blk;
};

struct Bin {            // one accumulation workgroup: chunk k of K of one region
  int32_t pair, region, k, pad;
};

// Pairs are binned and accumulated in groups of at most RM_GROUP_RECORDS
// record slots, reused from group to group, which bounds the record memory
// of very large launches.  (Groups small enough to keep the records in the
// last-level cache were measured slower: each launch then ends in a partial
// wave of workgroups.)
struct BinGroup {
  int32_t bb_begin, bb_end;    // binning blocks of the group
  int32_t bin_begin, bin_end;  // accumulation workgroups of the group
};

struct StepArgs {
  const ObjStatic* objs;
  ObjState* state;
  const KfDev* kfs;
  const StepObj* sobj;
  int32_t n_sobj;
  const Item* items;
  int32_t n_items;
  const Fin* fins;
  int32_t n_fins;
  RayRec* rays;
  int32_t n_rays;
  float2* e;            // [L][S] encodings (e_bf16: [L][S] uint32, a BF16 pair each)
  int e_bf16;           // encodings stored rounded to BF16 (the BF16 MLP reads nothing else)
  float2* de;           // [L][S] their adjoints
  int64_t S;            // samples = n_rays * N
  float* partials;      // n_items * RM_REC_STRIDE_NH(mlp_layers)
  float* wpack32;       // n_sobj * RM_WPACK
  uint16_t* wpack16;    // n_sobj * RM_WPACK
  uint32_t seed_lo, seed_hi;
  float lambda_depth, lambda_density;
  float lr, beta1, beta2, eps;
  int32_t mode;
  int32_t fuse_adam;    // training step: Adam applied where each gradient is complete
  int32_t mlp_layers;   // hidden layers of the density MLP (1..RM_MAX_MLP_LAYERS)
  const float* params_override; // single-object launches only
  float* grad_override;
  const float* adj_rgb;
  const float* adj_depth;
  const float* adj_tend;
  float* out_rgb;
  float* out_depth;
  float* out_tend;
  int32_t* dbg_kfuv;    // raygen: kf, u, v per ray (may be null)
  int32_t* dbg_cls;
  // binned scatter of the large levels
  const BinPair* bpairs;
  int32_t n_bpairs;
  const BinBlock* bblocks;
  int32_t n_bblocks;
  const Bin* bins;
  int32_t n_bins;
  int32_t bb_begin;     // this launch's first binning block / accumulation workgroup
  int32_t bin_begin;
  int32_t n_regions;    // bins over all pairs
  int32_t bin_max_R;    // most regions of one pair
  int32_t* bin_count;   // records per bin (zeroed by the gather kernel)
  float2* rec_val;      // records: values with the entry index in their low mantissa bits
};

// Launch helpers implemented in romap_kernels.hip.
hipError_t rm_launch_raygen(const StepArgs& a, int NS, hipStream_t st);
hipError_t rm_launch_encode_fwd(const StepArgs& a, int NS, int block, hipStream_t st);
hipError_t rm_launch_bin_scatter(const StepArgs& a, const BinGroup& g, int NS, hipStream_t st);
hipError_t rm_launch_bin_acc(const StepArgs& a, const BinGroup& g, hipStream_t st);
hipError_t rm_launch_pack(const StepArgs& a, int K1, hipStream_t st);
hipError_t rm_launch_field(const StepArgs& a, int NS, int K1, int prec, hipStream_t st);
hipError_t rm_launch_reduce(const StepArgs& a, hipStream_t st);
hipError_t rm_launch_bin_finish(const StepArgs& a, hipStream_t st);
hipError_t rm_launch_camera_rays(const StepArgs& a, int NS, const float* M, const float* c,
                                 float fx, float fy, float cx, float cy, int W, int pix0,
                                 hipStream_t st);
hipError_t rm_launch_user_rays(const StepArgs& a, int NS, const float* rays, hipStream_t st);
// marching cubes over a (res+1)^3 corner grid (x fastest)
#define RM_MC_SCAN 1024      /* cells per block of the count scan */
#define RM_MC_MAX_RES 160    /* res^3 <= 4096 scan blocks of RM_MC_SCAN */
struct MeshArgs {
  const float* grid;
  int res;
  float iso;
  float lo[3], hi[3];
  const int8_t* tris;       // [256][16] edge triples of each case
  const uint8_t* ntri;      // [256] triangles of each case
  const uint8_t* edge_a;    // [12] corners of each edge
  const uint8_t* edge_b;
  int* cnt;                 // res^3: triangles per cell, then in-block exclusive prefix
  int* bsum;                // per scan block: exclusive prefix of block totals; [nb] = total
  float* out;               // max_tris * 9
  int64_t max_tris;
  int world;                // apply x_w = R x + t
  float R[9], t[3];
};
hipError_t rm_launch_density_grid(const ObjStatic* objs, int obj, int nh, int res, float* grid,
                                  hipStream_t st);
hipError_t rm_launch_mc_count(const MeshArgs& m, hipStream_t st);
hipError_t rm_launch_mc_emit(const MeshArgs& m, hipStream_t st);
hipError_t rm_launch_query_density(const ObjStatic* objs, int obj, int nh, const float* xyz,
                                   int64_t n, float* sigma, hipStream_t st);
hipError_t rm_launch_debug_encode(const ObjStatic* objs, int obj, const float* p, int64_t n,
                                  uint32_t* idx, float* feat, hipStream_t st);
hipError_t rm_launch_fill(float* x, int64_t n, float v, hipStream_t st);
hipError_t rm_launch_occ_update(const ObjStatic* objs, int obj, int nh, uint32_t* bits,
                                float threshold, hipStream_t st);
hipError_t rm_launch_init(float* params, int64_t P_grid, int din, int nh, uint32_t k0,
                          uint32_t k1, hipStream_t st);
hipError_t rm_launch_debug_positions(const StepArgs& a, int NS, float* pos, hipStream_t st);
hipError_t rm_launch_reset_loss(const StepArgs& a, hipStream_t st);
hipError_t rm_launch_mfma_rate(int prec, int blocks, int iters, float* out, hipStream_t st);
double rm_mfma_rate_flops(int prec, int blocks, int iters);
