// romap_runtime.hip -- host side of libromap: the C ABI of include/romap.h.
//
// Owns the context: object registry (one hash-grid + MLP model per object
// instance, Sec. V), keyframe store with the view-angle rule of Eq. 5
// (Sec. V-A "Data"), per-step work lists covering every object of a step,
// hipGraph capture/replay of a step, the tile autotuner, and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/romap.h"
#include "romap_device.h"

// Scratch of the allocation-free entry point (romap_field_forward_noalloc):
// rays, encodings, packed weights and work tables of one call.  One copy per
// GPU, held until the process ends.  In host code `scratch` only names the
// symbol: its device address comes from hipGetSymbolAddress (scratch_address).
#define RM_SCRATCH_BYTES (size_t(64) << 20)
static __device__ __align__(256) char scratch[RM_SCRATCH_BYTES];

namespace {

std::string g_create_error;

// Ray-count limits.  One object's step writes at most 8 gradient records per
// sample and level, all of them possibly into one region of a small dense
// level: rays x samples <= 2^27 keeps that count, the region's bin counter
// and its capacity within int32.  Ray indices of a step are int32: at most
// 2^30 rays over the objects of one call.
constexpr int kMaxRaysPerObject = 1 << 22;
constexpr int64_t kMaxSamplesPerObject = int64_t(1) << 27;
constexpr int64_t kMaxRaysPerCall = int64_t(1) << 30;

bool ray_count_ok(int rays, int samples_per_ray) {
  return rays > 0 && rays <= kMaxRaysPerObject &&
         (int64_t)rays * samples_per_ray <= kMaxSamplesPerObject;
}

struct HostKf {
  romap_camera cam;
  uint8_t* d_rgb = nullptr;
  int32_t* d_mask = nullptr;
  float* d_depth = nullptr;
  std::vector<int32_t> h_mask;  // candidate rectangles of later-registered objects are not
                                // computed (keyframes join only objects registered before them)
};

struct HostObj {
  int id = 0, instance = 0, log2T = 0, active = 1;
  romap_box box{};
  int L = 0, din = 0, mlp_layers = 1;
  int64_t P = 0, P_grid = 0, P_alloc = 0;
  int64_t off[RM_MAX_LEVELS + 1]{};
  uint32_t N_l[RM_MAX_LEVELS]{}, T_l[RM_MAX_LEVELS]{};
  uint32_t hashed_mask = 0;
  float* d_block = nullptr;  // params | grad | m | v, P_alloc floats each
  std::vector<KfRef> kfs;
  KfRef* d_kfs = nullptr;
  size_t d_kfs_cap = 0;
  int64_t n_cand = 0;
  bool has_last = false;
  double last_centre[3]{};
  uint32_t* d_occ = nullptr;  // 64^3 occupancy bits
  bool occ_on = false;
  // the gradient buffer holds values (a training step needs it zero: its
  // Adam update is fused and only overflow or shared-region sums pass
  // through the buffer)
  bool grad_dirty = false;
};

struct Plan {                 // one launch: its objects, rays and work lists
  std::vector<StepObj> sobj;
  std::vector<Item> items;
  std::vector<Fin> fins;         // Adam work of regions summed by several workgroups
  std::vector<BinPair> bpairs;
  std::vector<BinBlock> bblocks;
  std::vector<Bin> bins;
  std::vector<BinGroup> bgroups;
  int64_t rec_size = 0;      // record slots of the largest group
  int64_t bin_regions = 0;  // regions over all pairs (bin_count entries)
  int n_rays = 0;
  int64_t S = 0;
  int rays_per_item = 8;
  int enc_block = 256;
  size_t off_sobj = 0, off_items = 0, off_fins = 0;  // in the device table arena (bytes)
  size_t off_bpairs = 0, off_bblocks = 0, off_bins = 0;
  // start of the plan's share of each scratch buffer (elements); nonzero for
  // the second of two plans whose steps run at the same time
  size_t so_rays = 0, so_e = 0, so_partials = 0, so_wpack = 0, so_bins = 0, so_rec = 0;
};

template <class T>
hipError_t grow(T** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return hipSuccess;
  size_t n = std::max(need, *cap * 2);
  if (n == 0) n = 1;
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return e;
    *p = nullptr;
  }
  *cap = 0;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e == hipSuccess) *cap = n;
  return e;
}

}  // namespace

struct romap_ctx {
  romap_config cfg{};
  int debug_bin_cap = 0;  // romap_debug_bin_capacity (0: sized capacity)
  int fixed_rpi = 8, fixed_blk = 256;  // launch shape without the autotuner (romap_debug_tiles)
  char* scratch_dev = nullptr;  // this device's `scratch` (set at creation)
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t stream2 = nullptr;   // second half of a split batched step
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // meshing: case tables (device) and scratch
  uint8_t* d_mc = nullptr;   // tris [256*16] int8 | ntri [256] | edge_a [12] | edge_b [12]
  float* d_mgrid = nullptr;
  size_t cap_mgrid = 0;
  int* d_mcnt = nullptr;
  size_t cap_mcnt = 0;
  int* d_mbsum = nullptr;
  float* d_mtris = nullptr;
  size_t cap_mtris = 0;
  std::vector<HostObj> objs;
  std::vector<HostKf> kfs;
  ObjStatic* d_objs = nullptr;
  size_t cap_objs = 0;
  ObjState* d_state = nullptr;
  size_t cap_state = 0;
  KfDev* d_kfdev = nullptr;
  size_t cap_kfdev = 0;
  // scratch of a step
  RayRec* d_rays = nullptr;
  size_t cap_rays = 0;
  float2* d_e = nullptr;
  float2* d_de = nullptr;
  size_t cap_e = 0, cap_de = 0;
  float* d_partials = nullptr;
  size_t cap_partials = 0;
  float* d_wpack32 = nullptr;
  uint16_t* d_wpack16 = nullptr;
  size_t cap_w32 = 0, cap_w16 = 0;
  char* d_tables = nullptr;
  size_t cap_tables = 0;
  int32_t* d_bin_count = nullptr;
  size_t cap_bin_count = 0;
  float2* d_rec_val = nullptr;
  size_t cap_rec_val = 0;
  // graph of the last batched step
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gsig;
  // autotuner results keyed by the work signature
  std::map<std::vector<int64_t>, std::pair<int, int>> tuned;
  // per-kernel timing of the last profiled train call
  std::vector<hipEvent_t> pev;  // event pool of the kernel timing (profile_phases)
  std::vector<int> pev_phase;    // phase that ends at each recorded event (-1: start)
  int pev_n = 0;                 // events recorded in the current step
  double phase_ms[ROMAP_N_PHASES] = {};
  double records_sum = 0;        // gradient records of the profiled steps
  int phase_steps = 0;
  std::string err;
};

namespace {

romap_status fail(romap_ctx* c, romap_status code, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, ROMAP_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define HIPALLOC(ctx, expr)                                                                \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation)                      \
      return fail(ctx, ROMAP_E_OUT_OF_MEMORY, std::string(#expr) + ": out of memory");     \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, ROMAP_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

bool is_fin(float x) { return std::isfinite(x); }

// Level table of the hash encoding: N_l = floor(N_min b^l + 1e-6) with
// b = exp((ln N_max - ln N_min)/(L - 1)); dense 1:1 when (N_l+1)^3 <= T.
void make_levels(const romap_config& cfg, int log2T, HostObj& o) {
  const int L = cfg.n_levels;
  double b = 1.0;
  if (L > 1) b = std::exp((std::log((double)cfg.max_res) - std::log((double)cfg.base_res)) / (double)(L - 1));
  const int64_t T = (int64_t)1 << log2T;
  int64_t off = 0;
  o.hashed_mask = 0;
  for (int l = 0; l < L; ++l) {
    const int N = L > 1 ? (int)std::floor((double)cfg.base_res * std::pow(b, (double)l) + 1e-6) : cfg.base_res;
    const int64_t dense = (int64_t)(N + 1) * (N + 1) * (N + 1);
    const bool hashed = dense > T;
    o.N_l[l] = (uint32_t)N;
    o.T_l[l] = (uint32_t)(hashed ? T : dense);
    if (hashed) o.hashed_mask |= 1u << l;
    o.off[l] = off;
    off += 2 * (int64_t)o.T_l[l];
  }
  o.off[L] = off;
  o.L = L;
  o.din = 2 * L;
  o.P_grid = off;
  o.mlp_layers = cfg.mlp_layers;
  o.P = off + (int64_t)RM_HIDDEN * o.din + (int64_t)(o.mlp_layers - 1) * RM_HH +
        RM_DOUT * RM_HIDDEN + RM_HIDDEN * RM_GEO + 3 * RM_HIDDEN;
  o.P_alloc = (o.P + 63) / 64 * 64;
}

// Camera -> object frame: with R = Rz(yaw), M = R^T R_wc, c = R^T (t_wc - t),
// computed in FP64 and rounded once.
void object_frame(const float* Twc, const romap_box& bx, float* M, float* c) {
  const double ct = std::cos((double)bx.yaw), st = std::sin((double)bx.yaw);
  for (int j = 0; j < 3; ++j) {
    const double r0 = (double)Twc[j], r1 = (double)Twc[4 + j], r2 = (double)Twc[8 + j];
    M[j] = (float)(ct * r0 + st * r1);
    M[3 + j] = (float)(-st * r0 + ct * r1);
    M[6 + j] = (float)r2;
  }
  const double dx = (double)Twc[3] - (double)bx.t[0];
  const double dy = (double)Twc[7] - (double)bx.t[1];
  const double dz = (double)Twc[11] - (double)bx.t[2];
  c[0] = (float)(ct * dx + st * dy);
  c[1] = (float)(-st * dx + ct * dy);
  c[2] = (float)dz;
}

ObjStatic to_static(const HostObj& o) {
  ObjStatic s{};
  s.params = o.d_block;
  s.grad = o.d_block + o.P_alloc;
  s.m = o.d_block + 2 * o.P_alloc;
  s.v = o.d_block + 3 * o.P_alloc;
  s.P = o.P;
  s.P_grid = o.P_grid;
  s.P_alloc = o.P_alloc;
  for (int l = 0; l <= RM_MAX_LEVELS; ++l) s.off[l] = o.off[l];
  for (int l = 0; l < RM_MAX_LEVELS; ++l) {
    s.N_l[l] = o.N_l[l];
    s.T_l[l] = o.T_l[l];
  }
  s.hashed_mask = o.hashed_mask;
  s.L = o.L;
  s.din = o.din;
  s.mlp_layers = o.mlp_layers;
  s.instance = o.instance;
  s.id = o.id;
  s.n_kf = (int)o.kfs.size();
  for (int k = 0; k < 3; ++k) s.half[k] = o.box.half[k];
  s.kfs = o.d_kfs;
  s.n_cand = o.n_cand;
  s.occ = o.occ_on ? o.d_occ : nullptr;
  return s;
}

romap_status upload_object(romap_ctx* c, int id) {
  HostObj& o = c->objs[id];
  if (!o.kfs.empty()) {
    if (o.kfs.size() > o.d_kfs_cap) {
      size_t cap = o.d_kfs_cap;
      HIPALLOC(c, grow(&o.d_kfs, &cap, o.kfs.size()));
      o.d_kfs_cap = cap;
    }
    HIPCHK(c, hipMemcpyAsync(o.d_kfs, o.kfs.data(), o.kfs.size() * sizeof(KfRef),
                             hipMemcpyHostToDevice, c->stream));
  }
  ObjStatic s = to_static(o);
  HIPCHK(c, hipMemcpyAsync(c->d_objs + id, &s, sizeof(s), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ROMAP_OK;
}

int K1_of(const romap_config& cfg) { return 2 * cfg.n_levels <= 16 ? 16 : 32; }

StepArgs base_args(romap_ctx* c) {
  StepArgs a{};
  a.objs = c->d_objs;
  a.state = c->d_state;
  a.kfs = c->d_kfdev;
  a.rays = c->d_rays;
  a.e = c->d_e;
  a.bin_count = c->d_bin_count;
  a.rec_val = c->d_rec_val;
  a.de = c->d_de;
  a.partials = c->d_partials;
  a.wpack32 = c->d_wpack32;
  a.wpack16 = c->d_wpack16;
  a.seed_lo = (uint32_t)c->cfg.seed;
  a.seed_hi = (uint32_t)(c->cfg.seed >> 32);
  a.lambda_depth = c->cfg.lambda_depth;
  a.lambda_density = c->cfg.lambda_density;
  a.lr = c->cfg.lr;
  a.beta1 = c->cfg.beta1;
  a.beta2 = c->cfg.beta2;
  a.eps = c->cfg.eps;
  a.mode = RM_MODE_TRAIN;
  a.mlp_layers = c->cfg.mlp_layers;
  a.e_bf16 = c->cfg.precision == ROMAP_PREC_BF16 ? 1 : 0;
  return a;
}

void build_items(Plan& p) {
  p.items.clear();
  for (size_t i = 0; i < p.sobj.size(); ++i) {
    StepObj& so = p.sobj[i];
    so.item_begin = (int)p.items.size();
    for (int r = 0; r < so.n_rays; r += p.rays_per_item) {
      Item it{};
      it.so = (int)i;
      it.ray_begin = so.ray_begin + r;
      it.n_rays = std::min(p.rays_per_item, so.n_rays - r);
      p.items.push_back(it);
    }
    so.item_end = (int)p.items.size();
  }
}

// Builds the work lists of a launch over (object, rays) pairs.
void build_plan(romap_ctx* c, const std::vector<std::pair<int, int>>& list, int rays_per_item,
                int enc_block, Plan& p) {
  p = Plan();
  p.rays_per_item = rays_per_item;
  p.enc_block = enc_block;
  int ray = 0;
  for (auto& pr : list) {
    StepObj so{};
    so.obj = pr.first;
    so.n_rays = pr.second;
    so.ray_begin = ray;
    ray += pr.second;
    p.sobj.push_back(so);
  }
  p.n_rays = ray;
  p.S = (int64_t)ray * c->cfg.samples_per_ray;
  build_items(p);
  // binned gradient scatter: every (object, level) pair
  const int NS = c->cfg.samples_per_ray;
  int64_t grp_rec = 0;  // record slots of the open group
  for (size_t i = 0; i < p.sobj.size(); ++i) {
    const HostObj& o = c->objs[p.sobj[i].obj];
    const int64_t So = (int64_t)p.sobj[i].n_rays * NS;
    for (int l = 0; l < o.L; ++l) {
      BinPair bp{};
      bp.so = (int)i;
      bp.l = l;
      bp.nb = (int)((So + RM_SCAT_WG - 1) / RM_SCAT_WG);
      bp.R = (int)((o.T_l[l] + RM_RB - 1) >> RM_RB_BITS);
      // corners shared by consecutive samples of a ray are merged on levels
      // with at most RM_MERGE_NUM / RM_MERGE_DEN cells per sample along a
      // box's side (on finer levels consecutive samples rarely touch)
      bp.merge = RM_MERGE_DEN * (int)o.N_l[l] <= RM_MERGE_NUM * NS;
      // records per region: 8 So / R on average (uniform hash, z-slabs of a
      // dense level); twice that plus a margin, a full bin falls back to atomics
      const int64_t expect = (8 * So + bp.R - 1) / bp.R;
      // hashed: near-uniform counts, the mean plus 8 standard deviations;
      // dense: regions are z-slabs, twice the mean (a full bin falls back to
      // atomics)
      const bool hashed = (o.hashed_mask >> l) & 1u;
      const int64_t want = hashed ? expect + 8 * (int64_t)std::ceil(std::sqrt((double)expect)) + 256
                                  : 2 * expect + 1024;
      bp.cap = (int)((std::min<int64_t>(want, 8 * So) + 3) & ~(int64_t)3);
      if (c->debug_bin_cap > 0) bp.cap = std::min(bp.cap, (c->debug_bin_cap + 3) & ~3);
      // workgroups per region: about RM_ACC_CHUNK records each, and at most
      // 2^(62 - RM_FX_BITS) / 2 per workgroup so no fixed-point sum can overflow
      const int64_t kmin = (bp.cap + ((int64_t)1 << (61 - RM_FX_BITS)) - 1) >> (61 - RM_FX_BITS);
      bp.K = (int)std::max<int64_t>(kmin, std::min<int64_t>(RM_ACC_MAXK, expect / RM_ACC_CHUNK));
      bp.K = std::max(bp.K, 1);
      const int64_t slots = (int64_t)bp.R * bp.cap;
      if (p.bgroups.empty() || (grp_rec > 0 && grp_rec + slots > RM_GROUP_RECORDS)) {
        const int nbb = (int)p.bblocks.size(), nbin = (int)p.bins.size();
        p.bgroups.push_back(BinGroup{nbb, nbb, nbin, nbin});
        grp_rec = 0;
      }
      bp.rec_base = grp_rec;  // record slots are reused from group to group
      grp_rec += slots;
      p.rec_size = std::max(p.rec_size, grp_rec);
      bp.bin_base = (int)p.bin_regions;
      p.bin_regions += bp.R;
      bp.s_begin = (int64_t)p.sobj[i].ray_begin * NS;
      bp.n_samples = So;
      const int pi = (int)p.bpairs.size();
      p.bpairs.push_back(bp);
      for (int b = 0; b < bp.nb; ++b) p.bblocks.push_back(BinBlock{pi, b});
      for (int r = 0; r < bp.R; ++r)
        for (int k = 0; k < bp.K; ++k) p.bins.push_back(Bin{pi, r, k, 0});
      if (bp.K > 1)
        for (int r = 0; r < bp.R; ++r) {
          const int64_t ne = std::min<int64_t>(RM_RB, (int64_t)o.T_l[l] - (int64_t)r * RM_RB);
          for (int sub = 0; sub * RM_FIN_WG < ne; ++sub) p.fins.push_back(Fin{pi, r, sub, 0});
        }
      p.bgroups.back().bb_end = (int)p.bblocks.size();
      p.bgroups.back().bin_end = (int)p.bins.size();
    }
  }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Makes sure the scratch buffers fit a set of plans, then uploads their
// work tables into the table arena.  Plans that run one after another share
// the scratch buffers; concurrent plans each get their own share of them.
romap_status stage_plans(romap_ctx* c, std::vector<Plan*> plans, bool concurrent = false) {
  size_t max_rays = 0, max_items = 0, max_sobj = 0, tab = 0, max_rec = 0, max_bins = 0;
  int64_t max_S = 0;
  const size_t L = (size_t)c->cfg.n_levels;
  const size_t nh = (size_t)c->cfg.mlp_layers;
  for (Plan* p : plans) {
    if (concurrent) {
      p->so_rays = max_rays;
      p->so_e = L * (size_t)max_S;
      p->so_partials = max_items * RM_REC_STRIDE_NH(nh);
      p->so_wpack = max_sobj * RM_WPACK_NH(nh);
      p->so_bins = max_bins;
      p->so_rec = max_rec;  // a multiple of 4: the bins' vector loads stay aligned
      max_rays += (size_t)p->n_rays;
      max_items += p->items.size();
      max_sobj += p->sobj.size();
      max_S += p->S;
      max_rec += (size_t)p->rec_size;
      max_bins += (size_t)p->bin_regions;
    } else {
      p->so_rays = p->so_e = p->so_partials = p->so_wpack = p->so_bins = p->so_rec = 0;
      max_rays = std::max(max_rays, (size_t)p->n_rays);
      max_items = std::max(max_items, p->items.size());
      max_sobj = std::max(max_sobj, p->sobj.size());
      max_S = std::max(max_S, p->S);
      max_rec = std::max(max_rec, (size_t)p->rec_size);
      max_bins = std::max(max_bins, (size_t)p->bin_regions);
    }
    p->off_sobj = tab;
    tab += align256(p->sobj.size() * sizeof(StepObj));
    p->off_items = tab;
    tab += align256(p->items.size() * sizeof(Item));
    p->off_fins = tab;
    tab += align256(p->fins.size() * sizeof(Fin));
    p->off_bpairs = tab;
    tab += align256(p->bpairs.size() * sizeof(BinPair));
    p->off_bblocks = tab;
    tab += align256(p->bblocks.size() * sizeof(BinBlock));
    p->off_bins = tab;
    tab += align256(p->bins.size() * sizeof(Bin));
  }
  auto regrow = [&](auto** ptr, size_t* cap, size_t need) -> hipError_t {
    if (need <= *cap) return hipSuccess;
    // a reallocation invalidates the captured graph
    if (c->gexec) {
      hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
      c->gsig.clear();
    }
    return grow(ptr, cap, need);
  };
  HIPALLOC(c, regrow(&c->d_rays, &c->cap_rays, std::max<size_t>(max_rays, 1)));
  HIPALLOC(c, regrow(&c->d_e, &c->cap_e, std::max<size_t>(L * (size_t)max_S, 1)));
  HIPALLOC(c, regrow(&c->d_de, &c->cap_de, std::max<size_t>(L * (size_t)max_S, 1)));
  HIPALLOC(c, regrow(&c->d_partials, &c->cap_partials,
                     std::max<size_t>(max_items * RM_REC_STRIDE_NH(nh), 1)));
  HIPALLOC(c, regrow(&c->d_wpack32, &c->cap_w32, std::max<size_t>(max_sobj * RM_WPACK_NH(nh), 1)));
  HIPALLOC(c, regrow(&c->d_wpack16, &c->cap_w16, std::max<size_t>(max_sobj * RM_WPACK_NH(nh), 1)));
  HIPALLOC(c, regrow(&c->d_tables, &c->cap_tables, std::max<size_t>(tab, 256)));
  HIPALLOC(c, regrow(&c->d_bin_count, &c->cap_bin_count, std::max<size_t>(max_bins, 1)));
  HIPALLOC(c, regrow(&c->d_rec_val, &c->cap_rec_val, std::max<size_t>(max_rec, 1)));
  std::vector<char> h(tab);
  for (Plan* p : plans) {
    if (!p->sobj.empty()) std::memcpy(h.data() + p->off_sobj, p->sobj.data(), p->sobj.size() * sizeof(StepObj));
    if (!p->items.empty()) std::memcpy(h.data() + p->off_items, p->items.data(), p->items.size() * sizeof(Item));
    if (!p->fins.empty()) std::memcpy(h.data() + p->off_fins, p->fins.data(), p->fins.size() * sizeof(Fin));
    if (!p->bpairs.empty()) std::memcpy(h.data() + p->off_bpairs, p->bpairs.data(), p->bpairs.size() * sizeof(BinPair));
    if (!p->bblocks.empty()) std::memcpy(h.data() + p->off_bblocks, p->bblocks.data(), p->bblocks.size() * sizeof(BinBlock));
    if (!p->bins.empty()) std::memcpy(h.data() + p->off_bins, p->bins.data(), p->bins.size() * sizeof(Bin));
  }
  if (tab) HIPCHK(c, hipMemcpyAsync(c->d_tables, h.data(), tab, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ROMAP_OK;
}

StepArgs plan_args(romap_ctx* c, const Plan& p) {
  StepArgs a = base_args(c);
  a.sobj = (const StepObj*)(c->d_tables + p.off_sobj);
  a.n_sobj = (int)p.sobj.size();
  a.items = (const Item*)(c->d_tables + p.off_items);
  a.n_items = (int)p.items.size();
  a.fins = (const Fin*)(c->d_tables + p.off_fins);
  a.n_fins = (int)p.fins.size();
  a.n_rays = p.n_rays;
  a.S = p.S;
  a.bpairs = (const BinPair*)(c->d_tables + p.off_bpairs);
  a.n_bpairs = (int)p.bpairs.size();
  a.bblocks = (const BinBlock*)(c->d_tables + p.off_bblocks);
  a.n_bblocks = (int)p.bblocks.size();
  a.bins = (const Bin*)(c->d_tables + p.off_bins);
  a.n_bins = (int)p.bins.size();
  a.rays = c->d_rays + p.so_rays;
  a.e = c->d_e + p.so_e;
  a.de = c->d_de + p.so_e;
  a.partials = c->d_partials + p.so_partials;
  a.wpack32 = c->d_wpack32 + p.so_wpack;
  a.wpack16 = c->d_wpack16 + p.so_wpack;
  a.bin_count = c->d_bin_count + p.so_bins;
  a.rec_val = c->d_rec_val + p.so_rec;
  a.n_regions = (int)p.bin_regions;
  a.bin_max_R = 0;
  for (const BinPair& bp : p.bpairs) a.bin_max_R = std::max(a.bin_max_R, bp.R);
  return a;
}

// One training step of every object of a plan (the hot path).  ev: null, or
// ROMAP_N_PHASES + 1 events recorded between the kernels.
// Records a timing event on the context stream; ph is the phase of the
// kernel launched just before it (-1 at the start of a step).
hipError_t mark_phase(romap_ctx* c, int ph) {
  if (c->pev_n == (int)c->pev.size()) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    c->pev.push_back(ev);
    c->pev_phase.push_back(-1);
  }
  c->pev_phase[c->pev_n] = ph;
  return hipEventRecord(c->pev[c->pev_n++], c->stream);
}

hipError_t enqueue_step(romap_ctx* c, const Plan& p, const StepArgs& a0, bool adam,
                        bool prof = false, hipStream_t st = nullptr, hipEvent_t ev_mid = nullptr,
                        int mid_phase = -1) {
  const int NS = c->cfg.samples_per_ray, K1 = K1_of(c->cfg);
  if (!st) st = c->stream;
  StepArgs a = a0;
  a.fuse_adam = adam ? 1 : 0;
  hipError_t e;
#define RM_MARK(ph) \
  if (prof && (e = mark_phase(c, ph)) != hipSuccess) return e;
  RM_MARK(-1);
  if ((e = rm_launch_raygen(a, NS, st)) != hipSuccess) return e;
  RM_MARK(ROMAP_PHASE_RAYGEN);
  if ((e = rm_launch_encode_fwd(a, NS, p.enc_block, st)) != hipSuccess) return e;
  RM_MARK(ROMAP_PHASE_ENCODE);
  if (ev_mid && mid_phase == ROMAP_PHASE_ENCODE && (e = hipEventRecord(ev_mid, st)) != hipSuccess)
    return e;
  if ((e = rm_launch_pack(a, K1, st)) != hipSuccess) return e;
  RM_MARK(ROMAP_PHASE_PACK);
  if ((e = rm_launch_field(a, NS, K1, c->cfg.precision, st)) != hipSuccess) return e;
  RM_MARK(ROMAP_PHASE_FIELD);
  if ((e = rm_launch_reduce(a, st)) != hipSuccess) return e;
  RM_MARK(ROMAP_PHASE_REDUCE);
  for (const BinGroup& g : p.bgroups) {
    if ((e = rm_launch_bin_scatter(a, g, NS, st)) != hipSuccess) return e;
    RM_MARK(ROMAP_PHASE_BIN_SCATTER);
    if ((e = rm_launch_bin_acc(a, g, st)) != hipSuccess) return e;
    RM_MARK(ROMAP_PHASE_BIN_ACC);
  }
  if ((e = rm_launch_bin_finish(a, st)) != hipSuccess) return e;
  RM_MARK(ROMAP_PHASE_BIN_FINISH);
#undef RM_MARK
  return hipSuccess;
}

// One step of two plans at the same time: the second on the context's second
// stream, joined back into the context stream (also under graph capture).
// Their objects differ and each has its own scratch, so the two only share
// the device.  The second group starts once the first has passed its
// gather, so that the groups run different phases at any time: the first
// group's latency-bound MLP kernel overlaps the second's bandwidth-bound
// gather, and so on down the step (measured on the 24-object workload:
// 1.898 ms per step with both groups started together, 1.816 with the
// offset; waiting for the first group's MLP instead: 1.877).
// `steps` steps in a row: each group's next step waits only for its own
// previous one (the groups' objects and scratch are disjoint), and the
// second group's step k for the first group's gather of step k; the groups
// join once at the end.  Eager steps use steps = 1; a captured graph holds
// RM_GRAPH_STEPS of them, so the first group does not wait at every step for
// the second group's tail.
hipError_t enqueue_pair(romap_ctx* c, const Plan* p, const StepArgs* a, int steps = 1) {
  hipError_t e;
  for (int k = 0; k < steps; ++k) {
    if ((e = enqueue_step(c, p[0], a[0], true, false, c->stream, c->ev_fork,
                          ROMAP_PHASE_ENCODE)) != hipSuccess)
      return e;
    if ((e = hipStreamWaitEvent(c->stream2, c->ev_fork, 0)) != hipSuccess) return e;
    if ((e = enqueue_step(c, p[1], a[1], true, false, c->stream2)) != hipSuccess) return e;
  }
  if ((e = hipEventRecord(c->ev_join, c->stream2)) != hipSuccess) return e;
  return hipStreamWaitEvent(c->stream, c->ev_join, 0);
}

// Splits a batched step's objects in two groups whose work (rays x samples x
// levels of gathers, records and MLP, plus the table's Adam bytes) is about
// RM_SPLIT_SHARE and the rest; each group keeps the list order.
void split_list(romap_ctx* c, const std::vector<std::pair<int, int>>& list,
                std::vector<std::pair<int, int>> half[2]) {
  const double per_sample = 200.0 * c->cfg.n_levels;  // bytes moved per sample (about)
  std::vector<std::pair<double, size_t>> cost;
  for (size_t i = 0; i < list.size(); ++i) {
    const HostObj& o = c->objs[list[i].first];
    cost.push_back({(double)list[i].second * c->cfg.samples_per_ray * per_sample +
                        24.0 * (double)o.P_grid, i});
  }
  std::sort(cost.begin(), cost.end(), [](const auto& x, const auto& y) {
    return x.first > y.first || (x.first == y.first && x.second < y.second);
  });
  std::vector<int> side(list.size(), 0);
  double w[2] = {0.0, 0.0};
  const double share[2] = {RM_SPLIT_SHARE, 1.0 - RM_SPLIT_SHARE};
  for (auto& cs : cost) {
    const int h = w[1] / share[1] < w[0] / share[0] ? 1 : 0;
    side[cs.second] = h;
    w[h] += cs.first;
  }
  half[0].clear();
  half[1].clear();
  for (size_t i = 0; i < list.size(); ++i) half[side[i]].push_back(list[i]);
}

// Adds the gradient records the step just run wrote into its bins (the
// binning kernel's fill counters, clamped at each bin's capacity).
romap_status count_records(romap_ctx* c, const Plan& p) {
  if (p.bin_regions == 0) return ROMAP_OK;
  std::vector<int32_t> cnt((size_t)p.bin_regions);
  HIPCHK(c, hipMemcpyAsync(cnt.data(), c->d_bin_count + p.so_bins, cnt.size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (const BinPair& bp : p.bpairs)
    for (int r = 0; r < bp.R; ++r) c->records_sum += std::min(cnt[bp.bin_base + r], bp.cap);
  return ROMAP_OK;
}

// Adds the kernel durations of the step whose events were just recorded:
// the time between two consecutive events belongs to the phase of the later.
hipError_t accumulate_phases(romap_ctx* c) {
  if (c->pev_n == 0) return hipSuccess;
  hipError_t e = hipEventSynchronize(c->pev[c->pev_n - 1]);
  if (e != hipSuccess) return e;
  for (int i = 1; i < c->pev_n; ++i) {
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, c->pev[i - 1], c->pev[i])) != hipSuccess) return e;
    c->phase_ms[c->pev_phase[i]] += ms;
  }
  c->pev_n = 0;
  return hipSuccess;
}

std::vector<int64_t> signature(romap_ctx* c, const std::vector<std::pair<int, int>>& list) {
  std::vector<int64_t> s = {c->cfg.samples_per_ray, c->cfg.n_levels, c->cfg.precision};
  for (auto& pr : list) {
    s.push_back(pr.first);
    s.push_back(pr.second);
  }
  return s;
}

// Tile autotuner: times the fused field kernel plus the record reduction for
// each ray-tile size, and the encoding gather for each block size, on the
// real work list; keeps the fastest.  Only scratch buffers and the gradient
// buffer's MLP part (rewritten by every step) are written.
romap_status autotune(romap_ctx* c, const std::vector<std::pair<int, int>>& list, int* rpi,
                      int* blk) {
  auto key = signature(c, list);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    *rpi = it->second.first;
    *blk = it->second.second;
    return ROMAP_OK;
  }
  const int NS = c->cfg.samples_per_ray, L = c->cfg.n_levels, K1 = K1_of(c->cfg);
  const int cands[] = {4, 8, 16, 32};
  const int blocks[] = {128, 256, 512};
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  float best = 1e30f;
  int best_rpi = 8, best_blk = 256;
  for (int cand : cands) {
    Plan p;
    build_plan(c, list, cand, 256, p);
    romap_status st = stage_plans(c, {&p});
    if (st != ROMAP_OK) return st;
    StepArgs a = plan_args(c, p);
    HIPCHK(c, rm_launch_raygen(a, NS, c->stream));
    HIPCHK(c, rm_launch_encode_fwd(a, NS, 256, c->stream));
    HIPCHK(c, rm_launch_pack(a, K1, c->stream));
    StepArgs ar = a;  // the reduce only sums the records here: no loss, no Adam
    ar.mode = RM_MODE_ADJOINT;
    HIPCHK(c, rm_launch_field(a, NS, K1, c->cfg.precision, c->stream));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < 3; ++r) {
      HIPCHK(c, rm_launch_field(a, NS, K1, c->cfg.precision, c->stream));
      HIPCHK(c, rm_launch_reduce(ar, c->stream));
    }
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      best_rpi = cand;
    }
    if (cand == cands[0]) {
      float bb = 1e30f;
      for (int blk_c : blocks) {
        HIPCHK(c, rm_launch_encode_fwd(a, NS, blk_c, c->stream));
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int r = 0; r < 3; ++r) HIPCHK(c, rm_launch_encode_fwd(a, NS, blk_c, c->stream));
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        if (ms < bb) {
          bb = ms;
          best_blk = blk_c;
        }
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  for (auto& pr : list) c->objs[pr.first].grad_dirty = true;  // the reduce wrote MLP gradients
  c->tuned[key] = {best_rpi, best_blk};
  *rpi = best_rpi;
  *blk = best_blk;
  return ROMAP_OK;
}

// Device address of the current device's `scratch`, looked up once per
// device (each GPU holds its own copy of the array at its own address).
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_at;

hipError_t scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_at.find(dev);
  if (it == g_scratch_at.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = g_scratch_at.emplace(dev, static_cast<char*>(p)).first;
  }
  *out = it->second;
  return hipSuccess;
}

romap_status check_object(romap_ctx* c, int32_t id) {
  if (id < 0 || id >= (int32_t)c->objs.size())
    return fail(c, ROMAP_E_NOT_FOUND, "unknown object id " + std::to_string(id));
  return ROMAP_OK;
}

romap_status validate_camera(romap_ctx* c, const romap_camera* cam) {
  if (!cam) return fail(c, ROMAP_E_INVALID_ARG, "camera is NULL");
  if (cam->width <= 0 || cam->height <= 0 || (int64_t)cam->width * cam->height > (1 << 26))
    return fail(c, ROMAP_E_INVALID_ARG, "bad image size");
  if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f) || !is_fin(cam->fx) || !is_fin(cam->fy) ||
      !is_fin(cam->cx) || !is_fin(cam->cy))
    return fail(c, ROMAP_E_INVALID_ARG, "bad intrinsics");
  for (int k = 0; k < 12; ++k)
    if (!is_fin(cam->T_wc[k])) return fail(c, ROMAP_E_INVALID_ARG, "non-finite pose");
  return ROMAP_OK;
}

romap_status read_losses(romap_ctx* c, const Plan& p, std::vector<float>* per_obj, int* n_nan) {
  std::vector<ObjState> st(c->objs.size());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(st.data(), c->d_state, st.size() * sizeof(ObjState), hipMemcpyDeviceToHost));
  per_obj->clear();
  *n_nan = 0;
  for (auto& so : p.sobj) {
    const ObjState& s = st[so.obj];
    const float l = s.n_loss ? s.loss_acc / (float)s.n_loss : 0.0f;
    if (!std::isfinite(l)) ++*n_nan;
    per_obj->push_back(l);
  }
  return ROMAP_OK;
}

romap_status resolve_list(romap_ctx* c, const int32_t* ids, int32_t n, const int32_t* rays,
                          std::vector<std::pair<int, int>>& list) {
  list.clear();
  if (ids) {
    if (n < 0) return fail(c, ROMAP_E_INVALID_ARG, "negative object count");
    for (int i = 0; i < n; ++i) {
      romap_status s = check_object(c, ids[i]);
      if (s != ROMAP_OK) return s;
      for (int j = 0; j < i; ++j)
        if (ids[j] == ids[i]) return fail(c, ROMAP_E_INVALID_ARG, "object listed twice");
      const int b = rays ? rays[i] : c->cfg.rays_per_step;
      if (!ray_count_ok(b, c->cfg.samples_per_ray))
        return fail(c, ROMAP_E_INVALID_ARG, "bad ray count");
      list.push_back({ids[i], b});
    }
  } else {
    int k = 0;
    for (auto& o : c->objs) {
      if (!o.active) continue;
      const int b = rays ? rays[k] : c->cfg.rays_per_step;
      if (!ray_count_ok(b, c->cfg.samples_per_ray))
        return fail(c, ROMAP_E_INVALID_ARG, "bad ray count");
      list.push_back({o.id, b});
      ++k;
    }
  }
  int64_t total = 0;
  for (auto& pr : list) total += pr.second;
  if (total > kMaxRaysPerCall) return fail(c, ROMAP_E_INVALID_ARG, "too many rays in one call");
  for (auto& pr : list)
    if (c->objs[pr.first].kfs.empty())
      return fail(c, ROMAP_E_STATE, "object " + std::to_string(pr.first) + " has no keyframe");
  return ROMAP_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

romap_status romap_default_config(romap_config* cfg) {
  if (!cfg) return ROMAP_E_INVALID_ARG;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n_levels = 16;
  cfg->base_res = 16;
  cfg->max_res = 1024;
  cfg->log2_table_size = 19;
  cfg->samples_per_ray = 64;
  cfg->rays_per_step = 4096;
  cfg->lr = 1e-2f;
  cfg->beta1 = 0.9f;
  cfg->beta2 = 0.99f;
  cfg->eps = 1e-15f;
  cfg->lambda_depth = 0.5f;
  cfg->lambda_density = 0.01f;
  cfg->alpha_deg = 25.0f;
  cfg->bbox_margin_pct = 10;
  cfg->precision = ROMAP_PREC_FP32;
  cfg->batch_mode = ROMAP_BATCH_ALL;
  cfg->use_graph = 1;
  cfg->autotune = 1;
  cfg->profile_phases = 0;
  cfg->mlp_layers = 1;
  cfg->streams = 2;
  cfg->seed = 0;
  return ROMAP_OK;
}

const char* romap_last_error(const romap_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

romap_status romap_create(const romap_config* cfg, void* hip_stream, romap_ctx** out) {
  if (!cfg || !out) return fail(nullptr, ROMAP_E_INVALID_ARG, "NULL argument");
  const romap_config& k = *cfg;
  if (k.n_levels < 1 || k.n_levels > 16) return fail(nullptr, ROMAP_E_INVALID_ARG, "n_levels must be 1..16");
  if (k.base_res < 1 || k.max_res < k.base_res || k.max_res > (1 << 16))
    return fail(nullptr, ROMAP_E_INVALID_ARG, "bad resolutions");
  if (k.log2_table_size < 8 || k.log2_table_size > 24)
    return fail(nullptr, ROMAP_E_INVALID_ARG, "log2_table_size must be 8..24");
  if (k.samples_per_ray != 32 && k.samples_per_ray != 64 && k.samples_per_ray != 128)
    return fail(nullptr, ROMAP_E_INVALID_ARG, "samples_per_ray must be 32, 64 or 128");
  if (k.mlp_layers < 1 || k.mlp_layers > RM_MAX_MLP_LAYERS)
    return fail(nullptr, ROMAP_E_INVALID_ARG, "mlp_layers must be 1..3");
  if (k.streams != 1 && k.streams != 2) return fail(nullptr, ROMAP_E_INVALID_ARG, "streams must be 1 or 2");
  if (k.use_graph < 0 || k.use_graph > 2) return fail(nullptr, ROMAP_E_INVALID_ARG, "use_graph must be 0, 1 or 2");
  if (!ray_count_ok(k.rays_per_step, k.samples_per_ray))
    return fail(nullptr, ROMAP_E_INVALID_ARG, "bad rays_per_step");
  if (!(k.lr > 0.0f) || !(k.beta1 >= 0.0f && k.beta1 < 1.0f) || !(k.beta2 >= 0.0f && k.beta2 < 1.0f) ||
      !(k.eps >= 0.0f) || !is_fin(k.lr))
    return fail(nullptr, ROMAP_E_INVALID_ARG, "bad Adam hyperparameters");
  if (!(k.lambda_depth >= 0.0f) || !(k.lambda_density >= 0.0f) || !is_fin(k.lambda_depth) ||
      !is_fin(k.lambda_density))
    return fail(nullptr, ROMAP_E_INVALID_ARG, "bad loss weights");
  if (!(k.alpha_deg >= 0.0f && k.alpha_deg <= 180.0f)) return fail(nullptr, ROMAP_E_INVALID_ARG, "bad alpha_deg");
  if (k.bbox_margin_pct < 0 || k.bbox_margin_pct > 100) return fail(nullptr, ROMAP_E_INVALID_ARG, "bad margin");
  if (k.precision != ROMAP_PREC_FP32 && k.precision != ROMAP_PREC_BF16)
    return fail(nullptr, ROMAP_E_INVALID_ARG, "bad precision");
  if (k.batch_mode != ROMAP_BATCH_ALL && k.batch_mode != ROMAP_BATCH_PER_OBJECT)
    return fail(nullptr, ROMAP_E_INVALID_ARG, "bad batch_mode");
  romap_ctx* c = new romap_ctx();
  c->cfg = k;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, ROMAP_E_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  const hipError_t se = scratch_address(&c->scratch_dev);
  if (se != hipSuccess) {
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
    return fail(nullptr, ROMAP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(se));
  }
  *out = c;
  return ROMAP_OK;
}

romap_status romap_destroy(romap_ctx* c) {
  if (!c) return ROMAP_E_INVALID_ARG;
  hipStreamSynchronize(c->stream);
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->stream2) {
    hipStreamSynchronize(c->stream2);
    hipStreamDestroy(c->stream2);
    hipEventDestroy(c->ev_fork);
    hipEventDestroy(c->ev_join);
  }
  for (hipEvent_t ev : c->pev) hipEventDestroy(ev);
  for (auto& o : c->objs) {
    hipFree(o.d_block);
    hipFree(o.d_kfs);
    hipFree(o.d_occ);
  }
  for (auto& k : c->kfs) {
    hipFree(k.d_rgb);
    hipFree(k.d_mask);
    hipFree(k.d_depth);
  }
  hipFree(c->d_objs);
  hipFree(c->d_state);
  hipFree(c->d_kfdev);
  hipFree(c->d_rays);
  hipFree(c->d_e);
  hipFree(c->d_de);
  hipFree(c->d_partials);
  hipFree(c->d_wpack32);
  hipFree(c->d_wpack16);
  hipFree(c->d_tables);
  hipFree(c->d_bin_count);
  hipFree(c->d_mc);
  hipFree(c->d_mgrid);
  hipFree(c->d_mcnt);
  hipFree(c->d_mbsum);
  hipFree(c->d_mtris);
  hipFree(c->d_rec_val);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
  return ROMAP_OK;
}

romap_status romap_get_phase_times(romap_ctx* c, float* avg_ms, int32_t* n_steps) {
  if (!c || !avg_ms) return ROMAP_E_INVALID_ARG;
  for (int i = 0; i < ROMAP_N_PHASES; ++i)
    avg_ms[i] = c->phase_steps ? (float)(c->phase_ms[i] / c->phase_steps) : 0.0f;
  if (n_steps) *n_steps = c->phase_steps;
  return ROMAP_OK;
}

romap_status romap_get_step_records(romap_ctx* c, double* avg_records) {
  if (!c || !avg_records) return ROMAP_E_INVALID_ARG;
  *avg_records = c->phase_steps ? c->records_sum / c->phase_steps : 0.0;
  return ROMAP_OK;
}

romap_status romap_sync(romap_ctx* c) {
  if (!c) return ROMAP_E_INVALID_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ROMAP_OK;
}

romap_status romap_add_object(romap_ctx* c, int32_t instance_id, const romap_box* box,
                              int32_t log2_table_size, int32_t* object_id) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (!box) return fail(c, ROMAP_E_INVALID_ARG, "box is NULL");
  if (instance_id < 1) return fail(c, ROMAP_E_INVALID_ARG, "instance ids start at 1 (0 = background)");
  for (int k = 0; k < 3; ++k)
    if (!(box->half[k] > 0.0f) || !is_fin(box->half[k]) || !is_fin(box->t[k]))
      return fail(c, ROMAP_E_INVALID_ARG, "box centre must be finite and half extents > 0");
  if (!is_fin(box->yaw)) return fail(c, ROMAP_E_INVALID_ARG, "non-finite yaw");
  const int lt = log2_table_size == 0 ? c->cfg.log2_table_size : log2_table_size;
  if (lt < 8 || lt > 24) return fail(c, ROMAP_E_INVALID_ARG, "log2_table_size must be 8..24");
  for (auto& o : c->objs)
    if (o.instance == instance_id) return fail(c, ROMAP_E_INVALID_ARG, "instance already registered");
  HostObj o;
  o.id = (int)c->objs.size();
  o.instance = instance_id;
  o.log2T = lt;
  o.box = *box;
  make_levels(c->cfg, lt, o);
  // device tables first, so that a failure leaves no half-registered object
  {
    size_t cap = c->cap_objs;
    if (c->objs.size() + 1 > cap) {
      ObjStatic* nd = nullptr;
      const size_t ncap = std::max<size_t>(16, 2 * cap);
      HIPALLOC(c, hipMalloc((void**)&nd, ncap * sizeof(ObjStatic)));
      ObjState* ns = nullptr;
      hipError_t e = hipMalloc((void**)&ns, ncap * sizeof(ObjState));
      if (e != hipSuccess) {
        hipFree(nd);
        return fail(c, ROMAP_E_OUT_OF_MEMORY, "object table: out of memory");
      }
      HIPCHK(c, hipMemsetAsync(ns, 0, ncap * sizeof(ObjState), c->stream));
      if (c->d_objs) {
        HIPCHK(c, hipMemcpyAsync(nd, c->d_objs, c->objs.size() * sizeof(ObjStatic), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(ns, c->d_state, c->objs.size() * sizeof(ObjState), hipMemcpyDeviceToDevice, c->stream));
      }
      HIPCHK(c, hipStreamSynchronize(c->stream));
      hipFree(c->d_objs);
      hipFree(c->d_state);
      c->d_objs = nd;
      c->d_state = ns;
      c->cap_objs = c->cap_state = ncap;
      if (c->gexec) {
        hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
        c->gsig.clear();
      }
    }
  }
  HIPALLOC(c, hipMalloc((void**)&o.d_block, 4 * (size_t)o.P_alloc * sizeof(float)));
  hipError_t e = hipMemsetAsync(o.d_block, 0, 4 * (size_t)o.P_alloc * sizeof(float), c->stream);
  if (e == hipSuccess)
    e = rm_launch_init(o.d_block, o.P_grid, o.din, o.mlp_layers,
                       (uint32_t)c->cfg.seed ^ (uint32_t)o.id,
                       (uint32_t)(c->cfg.seed >> 32), c->stream);
  ObjState st0{};
  st0.bc1 = 1.0f;
  st0.bc2 = 1.0f;
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->d_state + o.id, &st0, sizeof(st0), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    hipFree(o.d_block);
    return fail(c, ROMAP_E_HIP, std::string("object init: ") + hipGetErrorString(e));
  }
  c->objs.push_back(o);
  romap_status s = upload_object(c, o.id);
  if (s != ROMAP_OK) return s;
  if (object_id) *object_id = o.id;
  return ROMAP_OK;
}

romap_status romap_set_object_active(romap_ctx* c, int32_t id, int32_t active) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  c->objs[id].active = active ? 1 : 0;
  return ROMAP_OK;
}

static const size_t kOccBytes = 64 * 64 * 64 / 8;

romap_status romap_set_occupancy(romap_ctx* c, int32_t id, const uint8_t* bits) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  HostObj& o = c->objs[id];
  if (!bits) {
    o.occ_on = false;
    return upload_object(c, id);
  }
  if (!o.d_occ) HIPALLOC(c, hipMalloc((void**)&o.d_occ, kOccBytes));
  HIPCHK(c, hipMemcpyAsync(o.d_occ, bits, kOccBytes, hipMemcpyHostToDevice, c->stream));
  o.occ_on = true;
  return upload_object(c, id);
}

romap_status romap_update_occupancy(romap_ctx* c, int32_t id, float threshold) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (!std::isfinite(threshold)) return fail(c, ROMAP_E_INVALID_ARG, "non-finite threshold");
  HostObj& o = c->objs[id];
  if (!o.d_occ) HIPALLOC(c, hipMalloc((void**)&o.d_occ, kOccBytes));
  HIPCHK(c, rm_launch_occ_update(c->d_objs, id, c->cfg.mlp_layers, o.d_occ, threshold, c->stream));
  o.occ_on = true;
  return upload_object(c, id);
}

romap_status romap_get_occupancy(romap_ctx* c, int32_t id, uint8_t* bits) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (!bits) return fail(c, ROMAP_E_INVALID_ARG, "bits is NULL");
  const HostObj& o = c->objs[id];
  if (!o.occ_on) return fail(c, ROMAP_E_STATE, "occupancy skipping is off for this object");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(bits, o.d_occ, kOccBytes, hipMemcpyDeviceToHost));
  return ROMAP_OK;
}

romap_status romap_get_object_info(romap_ctx* c, int32_t id, romap_object_info* info) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (!info) return fail(c, ROMAP_E_INVALID_ARG, "info is NULL");
  const HostObj& o = c->objs[id];
  ObjState st{};
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(&st, c->d_state + id, sizeof(st), hipMemcpyDeviceToHost));
  std::memset(info, 0, sizeof(*info));
  info->instance_id = o.instance;
  info->log2_table_size = o.log2T;
  info->n_grid_params = o.P_grid;
  info->n_mlp_params = o.P - o.P_grid;
  info->n_keyframes = (int)o.kfs.size();
  info->step = st.step;
  info->n_candidates = o.n_cand;
  info->active = o.active;
  for (int l = 0; l < o.L; ++l) {
    info->level_res[l] = (int)o.N_l[l];
    info->level_hashed[l] = (o.hashed_mask >> l) & 1;
  }
  return ROMAP_OK;
}

romap_status romap_add_keyframe(romap_ctx* c, const romap_camera* cam, const uint8_t* rgb,
                                const int32_t* mask, const float* depth_z, int32_t* keyframe_id,
                                int32_t* n_objects_accepted) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = validate_camera(c, cam);
  if (s != ROMAP_OK) return s;
  if (!rgb || !mask) return fail(c, ROMAP_E_INVALID_ARG, "rgb and mask are required");
  const int W = cam->width, H = cam->height;
  const size_t npix = (size_t)W * H;
  // which objects accept this keyframe (Eq. 5), decided before any side effect
  struct Acc {
    int obj;
    int rect[4];
  };
  std::vector<Acc> acc;
  const double tI[3] = {cam->T_wc[3], cam->T_wc[7], cam->T_wc[11]};
  // bounding boxes of every registered instance in one pass over the mask
  std::map<int32_t, int> slot;
  for (auto& o : c->objs) slot[o.instance] = o.id;
  std::vector<int> bx0(c->objs.size(), W), bx1(c->objs.size(), -1), by0(c->objs.size(), H),
      by1(c->objs.size(), -1);
  {
    int32_t last_inst = 0;
    int last_slot = -1;
    for (int y = 0; y < H; ++y) {
      const int32_t* row = mask + (int64_t)y * W;
      for (int x = 0; x < W; ++x) {
        const int32_t m = row[x];
        if (m == 0) continue;
        if (m != last_inst) {
          auto it = slot.find(m);
          last_inst = m;
          last_slot = it == slot.end() ? -1 : it->second;
        }
        if (last_slot < 0) continue;
        bx0[last_slot] = std::min(bx0[last_slot], x);
        bx1[last_slot] = std::max(bx1[last_slot], x);
        by0[last_slot] = std::min(by0[last_slot], y);
        by1[last_slot] = std::max(by1[last_slot], y);
      }
    }
  }
  for (auto& o : c->objs) {
    Acc a;
    if (bx1[o.id] < 0) continue;  // the object is not observed in this image
    {  // detection box: mask bounding box widened by margin_pct percent per side
      const int w0 = bx1[o.id] - bx0[o.id] + 1, h0 = by1[o.id] - by0[o.id] + 1;
      const int mx = (w0 * c->cfg.bbox_margin_pct + 99) / 100;
      const int my = (h0 * c->cfg.bbox_margin_pct + 99) / 100;
      const int x0 = std::max(0, bx0[o.id] - mx), y0 = std::max(0, by0[o.id] - my);
      const int x1 = std::min(W - 1, bx1[o.id] + mx), y1 = std::min(H - 1, by1[o.id] + my);
      a.rect[0] = x0;
      a.rect[1] = y0;
      a.rect[2] = x1 - x0 + 1;
      a.rect[3] = y1 - y0 + 1;
    }
    if (o.has_last) {
      double va[3], vb[3], dot = 0, na = 0, nb = 0;
      for (int k = 0; k < 3; ++k) {
        va[k] = o.last_centre[k] - (double)o.box.t[k];
        vb[k] = tI[k] - (double)o.box.t[k];
        dot += va[k] * vb[k];
        na += va[k] * va[k];
        nb += vb[k] * vb[k];
      }
      double cs = dot / (std::sqrt(na) * std::sqrt(nb));
      cs = std::max(-1.0, std::min(1.0, cs));
      const double alpha = std::acos(cs) * 180.0 / M_PI;
      if (!(alpha > (double)c->cfg.alpha_deg)) continue;
    }
    a.obj = o.id;
    acc.push_back(a);
  }
  HostKf kf;
  kf.cam = *cam;
  HIPALLOC(c, hipMalloc((void**)&kf.d_rgb, npix * 3));
  hipError_t e = hipMalloc((void**)&kf.d_mask, npix * sizeof(int32_t));
  if (e == hipSuccess && depth_z) e = hipMalloc((void**)&kf.d_depth, npix * sizeof(float));
  if (e == hipSuccess && c->kfs.size() + 1 > c->cap_kfdev) {
    KfDev* nd = nullptr;
    const size_t ncap = std::max<size_t>(64, 2 * c->cap_kfdev);
    e = hipMalloc((void**)&nd, ncap * sizeof(KfDev));
    if (e == hipSuccess && c->d_kfdev)
      e = hipMemcpy(nd, c->d_kfdev, c->kfs.size() * sizeof(KfDev), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) {
      hipStreamSynchronize(c->stream);
      hipFree(c->d_kfdev);
      c->d_kfdev = nd;
      c->cap_kfdev = ncap;
      if (c->gexec) {
        hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
        c->gsig.clear();
      }
    } else if (nd) {
      hipFree(nd);
    }
  }
  if (e != hipSuccess) {
    hipFree(kf.d_rgb);
    hipFree(kf.d_mask);
    hipFree(kf.d_depth);
    return fail(c, e == hipErrorOutOfMemory ? ROMAP_E_OUT_OF_MEMORY : ROMAP_E_HIP,
                std::string("keyframe allocation: ") + hipGetErrorString(e));
  }
  HIPCHK(c, hipMemcpyAsync(kf.d_rgb, rgb, npix * 3, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(kf.d_mask, mask, npix * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  if (depth_z)
    HIPCHK(c, hipMemcpyAsync(kf.d_depth, depth_z, npix * sizeof(float), hipMemcpyHostToDevice, c->stream));
  KfDev kd{};
  kd.rgb = kf.d_rgb;
  kd.mask = kf.d_mask;
  kd.depth = kf.d_depth;
  kd.W = W;
  kd.H = H;
  kd.fx = cam->fx;
  kd.fy = cam->fy;
  kd.cx = cam->cx;
  kd.cy = cam->cy;
  const int kid = (int)c->kfs.size();
  HIPCHK(c, hipMemcpyAsync(c->d_kfdev + kid, &kd, sizeof(kd), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->kfs.push_back(kf);
  for (auto& a : acc) {
    HostObj& o = c->objs[a.obj];
    KfRef r{};
    r.kf = kid;
    r.x0 = a.rect[0];
    r.y0 = a.rect[1];
    r.w = a.rect[2];
    r.h = a.rect[3];
    object_frame(cam->T_wc, o.box, r.M, r.c);
    r.cand_begin = o.n_cand;
    o.kfs.push_back(r);
    o.n_cand += (int64_t)r.w * r.h;
    o.has_last = true;
    for (int k = 0; k < 3; ++k) o.last_centre[k] = tI[k];
    s = upload_object(c, o.id);
    if (s != ROMAP_OK) return s;
  }
  if (keyframe_id) *keyframe_id = kid;
  if (n_objects_accepted) *n_objects_accepted = (int)acc.size();
  return ROMAP_OK;
}

// Steps held by one captured graph of a call of n_steps steps.
static int graph_steps(int n_steps) { return n_steps >= RM_GRAPH_STEPS ? RM_GRAPH_STEPS : 1; }

// The captured step graph is keyed by the objects, their ray counts, the
// tile choice, the work-table arena, the stream count and the steps it holds.
static std::vector<int64_t> graph_sig(romap_ctx* c, const std::vector<std::pair<int, int>>& list,
                                      int rpi, int blk, int steps) {
  std::vector<int64_t> sig = signature(c, list);
  sig.push_back(rpi);
  sig.push_back(blk);
  sig.push_back((int64_t)(uintptr_t)c->d_tables);
  sig.push_back(c->cfg.streams);
  sig.push_back(steps);
  return sig;
}

// A graph is used when it exists for this step already, or when the call
// replays it often enough to repay a capture (a few milliseconds); short
// calls with new shapes (a mapping stream's per-frame steps) run eagerly.
// use_graph = 2 captures on any call (a caller that warms up before timing).
static bool graph_pays(romap_ctx* c, const std::vector<std::pair<int, int>>& list, int rpi,
                       int blk, int n_steps) {
  if (c->cfg.use_graph == 2 || n_steps >= RM_GRAPH_MIN_STEPS) return true;
  return c->gexec && graph_sig(c, list, rpi, blk, graph_steps(n_steps)) == c->gsig;
}

romap_status romap_train(romap_ctx* c, const int32_t* ids, int32_t n, int32_t n_steps,
                         const int32_t* rays, romap_train_stats* stats) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (n_steps < 0) return fail(c, ROMAP_E_INVALID_ARG, "negative step count");
  std::vector<std::pair<int, int>> list;
  romap_status s = resolve_list(c, ids, n, rays, list);
  if (s != ROMAP_OK) return s;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (list.empty() || n_steps == 0) return ROMAP_OK;
  int rpi = c->fixed_rpi, blk = c->fixed_blk;
  if (c->cfg.autotune) {
    s = autotune(c, list, &rpi, &blk);
    if (s != ROMAP_OK) return s;
  }
  // a training step keeps the gradient buffer at zero; clear it where
  // romap_loss_and_grad, romap_set_params or the autotuner left values
  for (auto& pr : list) {
    HostObj& o = c->objs[pr.first];
    if (o.grad_dirty) {
      HIPCHK(c, rm_launch_fill(o.d_block + o.P_alloc, o.P_alloc, 0.0f, c->stream));
      o.grad_dirty = false;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
  }
  int64_t rays_total = 0;
  for (auto& pr : list) rays_total += pr.second;
  std::vector<float> losses;
  int n_nan = 0;
  Plan all;
  build_plan(c, list, rpi, blk, all);
  const bool prof = c->cfg.profile_phases != 0;
  // a batched step of two or more objects runs as two concurrent halves
  const bool split = c->cfg.batch_mode == ROMAP_BATCH_ALL && c->cfg.streams == 2 && !prof &&
                     list.size() >= 2;
  Plan half[2];
  if (split) {
    std::vector<std::pair<int, int>> hl[2];
    split_list(c, list, hl);
    build_plan(c, hl[0], rpi, blk, half[0]);
    build_plan(c, hl[1], rpi, blk, half[1]);
    if (!c->stream2) {
      HIPCHK(c, hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
      HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
      HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
  }
  if (prof) {
    c->pev_n = 0;
    c->records_sum = 0;
    for (int i = 0; i < ROMAP_N_PHASES; ++i) c->phase_ms[i] = 0.0;
    c->phase_steps = 0;
  }
  if (c->cfg.batch_mode == ROMAP_BATCH_ALL) {
    s = split ? stage_plans(c, {&half[0], &half[1]}, true) : stage_plans(c, {&all});
    if (s != ROMAP_OK) return s;
    StepArgs a = split ? StepArgs{} : plan_args(c, all);
    StepArgs ah[2];
    if (split) {
      ah[0] = plan_args(c, half[0]);
      ah[1] = plan_args(c, half[1]);
    }
    auto one_step = [&]() -> hipError_t {
      return split ? enqueue_pair(c, half, ah) : enqueue_step(c, all, a, true);
    };
    if (stats) {
      if (split) {
        HIPCHK(c, rm_launch_reset_loss(ah[0], c->stream));
        HIPCHK(c, rm_launch_reset_loss(ah[1], c->stream));
      } else {
        HIPCHK(c, rm_launch_reset_loss(a, c->stream));
      }
      HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    if (prof) {
      for (int i = 0; i < n_steps; ++i) {
        HIPCHK(c, enqueue_step(c, all, a, true, true));
        HIPCHK(c, accumulate_phases(c));
        s = count_records(c, all);
        if (s != ROMAP_OK) return s;
        ++c->phase_steps;
      }
    } else if (c->cfg.use_graph && graph_pays(c, list, rpi, blk, n_steps)) {
      const int G = graph_steps(n_steps);
      std::vector<int64_t> sig = graph_sig(c, list, rpi, blk, G);
      if (!c->gexec || sig != c->gsig) {
        if (c->gexec) {
          hipGraphExecDestroy(c->gexec);
          c->gexec = nullptr;
        }
        hipGraph_t graph;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        if (split)
          le = enqueue_pair(c, half, ah, G);
        else
          for (int k = 0; k < G && le == hipSuccess; ++k) le = enqueue_step(c, all, a, true);
        hipError_t ce = hipStreamEndCapture(c->stream, &graph);
        if (le != hipSuccess) return fail(c, ROMAP_E_HIP, std::string("capture: ") + hipGetErrorString(le));
        if (ce != hipSuccess) return fail(c, ROMAP_E_HIP, std::string("end capture: ") + hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ie != hipSuccess) {
          c->gexec = nullptr;
          return fail(c, ROMAP_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
        }
        c->gsig = sig;
      }
      int i = 0;
      for (; i + G <= n_steps; i += G) HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      for (; i < n_steps; ++i) HIPCHK(c, one_step());  // the remainder, eagerly
    } else {
      for (int i = 0; i < n_steps; ++i) HIPCHK(c, one_step());
    }
    if (stats) {
      HIPCHK(c, hipEventRecord(e1, c->stream));
      s = read_losses(c, all, &losses, &n_nan);  // per object, in list order
      if (s != ROMAP_OK) return s;
    }
  } else {
    // one launch per object per phase (the plain path)
    std::vector<Plan> plans(list.size());
    std::vector<Plan*> pp;
    for (size_t i = 0; i < list.size(); ++i) {
      build_plan(c, {list[i]}, rpi, blk, plans[i]);
      pp.push_back(&plans[i]);
    }
    s = stage_plans(c, pp);
    if (s != ROMAP_OK) return s;
    std::vector<StepArgs> args;
    for (auto& p : plans) args.push_back(plan_args(c, p));
    if (stats) {
      for (auto& a : args) HIPCHK(c, rm_launch_reset_loss(a, c->stream));
      HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    for (int i = 0; i < n_steps; ++i) {
      for (size_t k = 0; k < plans.size(); ++k) {
        HIPCHK(c, enqueue_step(c, plans[k], args[k], true, prof));
        if (prof) {
          HIPCHK(c, accumulate_phases(c));
          s = count_records(c, plans[k]);
          if (s != ROMAP_OK) return s;
        }
      }
      if (prof) ++c->phase_steps;
    }
    if (stats) {
      HIPCHK(c, hipEventRecord(e1, c->stream));
      losses.clear();
      for (auto& p : plans) {
        std::vector<float> l1;
        int nn = 0;
        s = read_losses(c, p, &l1, &nn);
        if (s != ROMAP_OK) return s;
        losses.insert(losses.end(), l1.begin(), l1.end());
        n_nan += nn;
      }
    }
  }
  if (stats) {
    float ms = 0.0f;
    HIPCHK(c, hipEventSynchronize(e1));
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    double sum = 0.0;
    for (float l : losses) sum += l;
    stats->loss_mean = losses.empty() ? 0.0f : (float)(sum / losses.size());
    stats->rays_trained = rays_total * n_steps;
    stats->seconds = ms * 1e-3f;
    stats->n_objects_nan = n_nan;
    if (n_nan) return fail(c, ROMAP_E_NUMERIC, std::to_string(n_nan) + " object(s) with non-finite loss");
  }
  return ROMAP_OK;
}

romap_status romap_loss_and_grad(romap_ctx* c, const int32_t* ids, int32_t n, const int32_t* rays,
                                 float* losses) {
  if (!c) return ROMAP_E_INVALID_ARG;
  std::vector<std::pair<int, int>> list;
  romap_status s = resolve_list(c, ids, n, rays, list);
  if (s != ROMAP_OK) return s;
  if (list.empty()) return ROMAP_OK;
  int rpi = c->fixed_rpi, blk = c->fixed_blk;  // the launch shape of a training step
  if (c->cfg.autotune) {
    s = autotune(c, list, &rpi, &blk);
    if (s != ROMAP_OK) return s;
  }
  Plan p;
  build_plan(c, list, rpi, blk, p);
  s = stage_plans(c, {&p});
  if (s != ROMAP_OK) return s;
  for (auto& pr : list) {
    const HostObj& o = c->objs[pr.first];
    HIPCHK(c, rm_launch_fill(o.d_block + o.P_alloc, o.P_alloc, 0.0f, c->stream));
  }
  StepArgs a = plan_args(c, p);
  HIPCHK(c, rm_launch_reset_loss(a, c->stream));
  HIPCHK(c, enqueue_step(c, p, a, false));
  for (auto& pr : list) c->objs[pr.first].grad_dirty = true;
  std::vector<float> l;
  int nn = 0;
  s = read_losses(c, p, &l, &nn);
  if (s != ROMAP_OK) return s;
  if (losses)
    for (size_t i = 0; i < l.size(); ++i) losses[i] = l[i];
  return ROMAP_OK;
}

romap_status romap_render(romap_ctx* c, int32_t id, const romap_camera* cam, float* rgb,
                          float* depth, float* opacity, int32_t on_device) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  s = validate_camera(c, cam);
  if (s != ROMAP_OK) return s;
  const HostObj& o = c->objs[id];
  const int W = cam->width, H = cam->height;
  const int64_t npix = (int64_t)W * H;
  float M[9], cc[3];
  object_frame(cam->T_wc, o.box, M, cc);
  float *d_rgb = nullptr, *d_depth = nullptr, *d_tend = nullptr;
  if (on_device) {
    d_rgb = rgb;
    d_depth = depth;
  } else {
    if (rgb) HIPALLOC(c, hipMalloc((void**)&d_rgb, npix * 3 * sizeof(float)));
    if (depth) HIPALLOC(c, hipMalloc((void**)&d_depth, npix * sizeof(float)));
  }
  if (opacity) HIPALLOC(c, hipMalloc((void**)&d_tend, npix * sizeof(float)));
  const int chunk = 32768;
  const int NS = c->cfg.samples_per_ray, L = c->cfg.n_levels, K1 = K1_of(c->cfg);
  for (int64_t p0 = 0; p0 < npix; p0 += chunk) {
    const int nr = (int)std::min<int64_t>(chunk, npix - p0);
    Plan p;
    build_plan(c, {{id, nr}}, 8, 256, p);
    p.fins.clear();  // forward only: no Adam, no gradient scatter (the
    p.bins.clear();  // sample blocks stay: the gather runs over them)
    p.bgroups.clear();
    p.rec_size = 0;
    p.bin_regions = 0;
    s = stage_plans(c, {&p});
    if (s != ROMAP_OK) return s;
    StepArgs a = plan_args(c, p);
    a.mode = RM_MODE_FORWARD;
    a.out_rgb = d_rgb ? d_rgb + 3 * p0 : nullptr;
    a.out_depth = d_depth ? d_depth + p0 : nullptr;
    a.out_tend = d_tend ? d_tend + p0 : nullptr;
    HIPCHK(c, rm_launch_camera_rays(a, NS, M, cc, cam->fx, cam->fy, cam->cx, cam->cy, W, (int)p0, c->stream));
    HIPCHK(c, rm_launch_encode_fwd(a, NS, 256, c->stream));
    HIPCHK(c, rm_launch_pack(a, K1, c->stream));
    HIPCHK(c, rm_launch_field(a, NS, K1, c->cfg.precision, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (!on_device) {
    if (rgb) HIPCHK(c, hipMemcpy(rgb, d_rgb, npix * 3 * sizeof(float), hipMemcpyDeviceToHost));
    if (depth) HIPCHK(c, hipMemcpy(depth, d_depth, npix * sizeof(float), hipMemcpyDeviceToHost));
    hipFree(d_rgb);
    hipFree(d_depth);
  }
  if (opacity) {
    std::vector<float> t(npix);
    HIPCHK(c, hipMemcpy(t.data(), d_tend, npix * sizeof(float), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < npix; ++i) t[i] = 1.0f - t[i];
    if (on_device)
      HIPCHK(c, hipMemcpy(opacity, t.data(), npix * sizeof(float), hipMemcpyHostToDevice));
    else
      std::memcpy(opacity, t.data(), npix * sizeof(float));
    hipFree(d_tend);
  }
  return ROMAP_OK;
}

// ---- object box from its point cloud (Sec. IV-B) --------------------------------

romap_status romap_box_from_points(const float* xyz, int64_t n, romap_box* box) {
  if (!xyz || n < 1 || !box) return ROMAP_E_INVALID_ARG;
  // Eq. 1: centre of the world-axis extremes
  double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
  double sx = 0, sy = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], (double)xyz[3 * i + k]);
      hi[k] = std::max(hi[k], (double)xyz[3 * i + k]);
    }
    sx += xyz[3 * i];
    sy += xyz[3 * i + 1];
  }
  double t[3];
  for (int k = 0; k < 3; ++k) t[k] = (lo[k] + hi[k]) / 2;
  // yaw: principal axis of the horizontal projection (second moments about
  // the mean), an axis without sign, folded into [-pi/2, pi/2)
  const double mx = sx / (double)n, my = sy / (double)n;
  double cxx = 0, cyy = 0, cxy = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double u = xyz[3 * i] - mx, w = xyz[3 * i + 1] - my;
    cxx += u * u;
    cyy += w * w;
    cxy += u * w;
  }
  const double PI = 3.14159265358979323846;
  double yaw = std::atan2(2 * cxy, cxx - cyy) / 2;
  if (yaw < -PI / 2) yaw += PI;
  if (yaw >= PI / 2) yaw -= PI;
  // Eq. 4: half the extent of the points in the object frame
  const double c = std::cos(yaw), s = std::sin(yaw);
  double olo[3] = {0, 0, 0}, ohi[3] = {0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    const double d[3] = {xyz[3 * i] - t[0], xyz[3 * i + 1] - t[1], xyz[3 * i + 2] - t[2]};
    const double q[3] = {c * d[0] + s * d[1], c * d[1] - s * d[0], d[2]};
    for (int k = 0; k < 3; ++k) {
      olo[k] = i ? std::min(olo[k], q[k]) : q[k];
      ohi[k] = i ? std::max(ohi[k], q[k]) : q[k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    box->t[k] = (float)t[k];
    box->half[k] = (float)((ohi[k] - olo[k]) / 2);
  }
  box->yaw = (float)yaw;
  return ROMAP_OK;
}

// ---- meshing (marching cubes) ------------------------------------------------

// Case table of marching cubes, derived from the cube's faces.  Corner c sits
// at (c&1, c>>1&1, c>>2&1); edges 0-3 run along x from corners 0,2,4,6, edges
// 4-7 along y from 0,1,4,5, edges 8-11 along z from 0,1,2,3; a corner is
// inside when its value exceeds iso.  Per case: the crossing edges of each
// face are joined in pairs (two crossings: the pair; four: each inside corner
// of the face cut off by its two edges), which closes them into loops; a
// loop is oriented so that its Newell normal over the edge midpoints points
// from the inside to the outside end of its first edge, rotated to start at
// its smallest edge, loops ordered by that edge, and each becomes a fan from
// its first vertex whose fan puts no triangle inside a cube face.
struct McTable {
  int8_t tris[256][16];
  uint8_t ntri[256];
  uint8_t ea[12], eb[12];
};

static void build_mc_table(McTable& T) {
  for (int e = 0; e < 12; ++e) {
    const int axis = e / 4, j = e % 4;
    // the corners with the axis bit clear, in increasing order
    int lows[4], n = 0;
    for (int c = 0; c < 8; ++c)
      if (!((c >> axis) & 1)) lows[n++] = c;
    T.ea[e] = (uint8_t)lows[j];
    T.eb[e] = (uint8_t)(lows[j] | (1 << axis));
  }
  auto edge_between = [&](int a, int b) {
    for (int e = 0; e < 12; ++e)
      if ((T.ea[e] == a && T.eb[e] == b) || (T.ea[e] == b && T.eb[e] == a)) return e;
    return -1;
  };
  // faces as corner cycles: fixed axis bit, cycle through the other two
  std::vector<std::array<int, 4>> faces;
  for (int axis = 0; axis < 3; ++axis)
    for (int side = 0; side < 2; ++side) {
      const int u = (axis + 1) % 3, w = (axis + 2) % 3;
      const int lo = std::min(u, w), hi = std::max(u, w);
      const int base = side << axis;
      faces.push_back({base, base | (1 << lo), base | (1 << lo) | (1 << hi), base | (1 << hi)});
    }
  auto on_face = [&](int e, const std::array<int, 4>& f) {
    int k = 0;
    for (int c : f) k += (c == T.ea[e]) + (c == T.eb[e]);
    return k == 2;
  };
  for (int m = 0; m < 256; ++m) {
    auto in = [&](int c) { return (m >> c) & 1; };
    std::vector<std::vector<int>> link(12);
    for (const auto& f : faces) {
      int side[4];
      std::vector<int> cross;
      for (int i = 0; i < 4; ++i) {
        side[i] = edge_between(f[i], f[(i + 1) % 4]);
        if (in(f[i]) != in(f[(i + 1) % 4])) cross.push_back(side[i]);
      }
      std::vector<std::pair<int, int>> pairs;
      if (cross.size() == 2) {
        pairs.push_back({cross[0], cross[1]});
      } else if (cross.size() == 4) {
        const int k0 = in(f[0]) ? 0 : 1;  // the face's inside corners: f[k0], f[k0 + 2]
        for (int k = k0; k < 4; k += 2) pairs.push_back({side[(k + 3) % 4], side[k]});
      }
      for (auto& pr : pairs) {
        link[pr.first].push_back(pr.second);
        link[pr.second].push_back(pr.first);
      }
    }
    std::vector<std::vector<int>> loops;
    std::vector<bool> seen(12, false);
    for (int e0 = 0; e0 < 12; ++e0) {
      if (link[e0].empty() || seen[e0]) continue;
      std::vector<int> lp{e0};
      seen[e0] = true;
      int prev = e0, cur = std::min(link[e0][0], link[e0][1]);
      while (cur != e0) {
        lp.push_back(cur);
        seen[cur] = true;
        const int nx = link[cur][0] == prev ? link[cur][1] : link[cur][0];
        prev = cur;
        cur = nx;
      }
      // orientation: Newell normal vs inside -> outside of the first edge
      double nrm[3] = {0, 0, 0};
      auto mid = [&](int e, int a) { return 0.5 * (((T.ea[e] >> a) & 1) + ((T.eb[e] >> a) & 1)); };
      const size_t L = lp.size();
      for (size_t i = 0; i < L; ++i) {
        const int p = lp[i], q = lp[(i + 1) % L];
        nrm[0] += (mid(p, 1) - mid(q, 1)) * (mid(p, 2) + mid(q, 2));
        nrm[1] += (mid(p, 2) - mid(q, 2)) * (mid(p, 0) + mid(q, 0));
        nrm[2] += (mid(p, 0) - mid(q, 0)) * (mid(p, 1) + mid(q, 1));
      }
      const int ci = in(T.ea[lp[0]]) ? T.ea[lp[0]] : T.eb[lp[0]];
      const int co = ci == T.ea[lp[0]] ? T.eb[lp[0]] : T.ea[lp[0]];
      double d = 0;
      for (int a = 0; a < 3; ++a) d += nrm[a] * (double)(((co >> a) & 1) - ((ci >> a) & 1));
      if (d < 0) std::reverse(lp.begin(), lp.end());
      std::rotate(lp.begin(), std::min_element(lp.begin(), lp.end()), lp.end());
      loops.push_back(lp);
    }
    std::sort(loops.begin(), loops.end(),
              [](const std::vector<int>& x, const std::vector<int>& y) { return x[0] < y[0]; });
    int nt = 0;
    for (const auto& lp : loops) {
      const int L = (int)lp.size();
      int apex = 0;
      for (int a0 = 0; a0 < L; ++a0) {
        bool flat = false;
        for (int i = 1; i + 1 < L && !flat; ++i)
          for (const auto& f : faces)
            if (on_face(lp[a0], f) && on_face(lp[(a0 + i) % L], f) && on_face(lp[(a0 + i + 1) % L], f))
              flat = true;
        if (!flat) {
          apex = a0;
          break;
        }
      }
      for (int i = 1; i + 1 < L; ++i, ++nt) {
        T.tris[m][3 * nt] = (int8_t)lp[apex];
        T.tris[m][3 * nt + 1] = (int8_t)lp[(apex + i) % L];
        T.tris[m][3 * nt + 2] = (int8_t)lp[(apex + i + 1) % L];
      }
    }
    for (int i = 3 * nt; i < 16; ++i) T.tris[m][i] = -1;
    T.ntri[m] = (uint8_t)nt;
  }
}

int32_t romap_mc_case(int32_t m, int8_t tris[16]) {
  static McTable T;
  static bool built = false;
  if (!built) {
    build_mc_table(T);
    built = true;
  }
  for (int i = 0; i < 16; ++i) tris[i] = T.tris[m & 255][i];
  return T.ntri[m & 255];
}

static romap_status mc_setup(romap_ctx* c, int res) {
  if (!c->d_mc) {
    McTable T;
    build_mc_table(T);
    std::vector<uint8_t> h(256 * 16 + 256 + 24);
    std::memcpy(h.data(), T.tris, 256 * 16);
    std::memcpy(h.data() + 4096, T.ntri, 256);
    std::memcpy(h.data() + 4352, T.ea, 12);
    std::memcpy(h.data() + 4364, T.eb, 12);
    HIPALLOC(c, hipMalloc((void**)&c->d_mc, h.size()));
    HIPALLOC(c, hipMalloc((void**)&c->d_mbsum, (RM_MC_MAX_RES * RM_MC_MAX_RES * RM_MC_MAX_RES /
                                                    RM_MC_SCAN + 2) * sizeof(int)));
    HIPCHK(c, hipMemcpy(c->d_mc, h.data(), h.size(), hipMemcpyHostToDevice));
  }
  const size_t n1 = (size_t)res + 1;
  HIPALLOC(c, grow(&c->d_mgrid, &c->cap_mgrid, n1 * n1 * n1));
  HIPALLOC(c, grow(&c->d_mcnt, &c->cap_mcnt, (size_t)res * res * res));
  return ROMAP_OK;
}

// Counts the triangles of m.grid and, if tris is given, writes up to max_tris
// of them (host or device buffer).
static romap_status mc_run(romap_ctx* c, MeshArgs& m, float* tris, int64_t max_tris,
                           int64_t* n_tris, int on_device) {
  m.tris = (const int8_t*)c->d_mc;
  m.ntri = c->d_mc + 4096;
  m.edge_a = c->d_mc + 4352;
  m.edge_b = c->d_mc + 4364;
  m.cnt = c->d_mcnt;
  m.bsum = c->d_mbsum;
  HIPCHK(c, rm_launch_mc_count(m, c->stream));
  const int64_t nc = (int64_t)m.res * m.res * m.res;
  const int nb = (int)((nc + RM_MC_SCAN - 1) / RM_MC_SCAN);
  int total = 0;
  HIPCHK(c, hipMemcpyAsync(&total, c->d_mbsum + nb, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (n_tris) *n_tris = total;
  const int64_t nw = std::min<int64_t>(total, max_tris);
  if (!tris || nw <= 0) return ROMAP_OK;
  m.max_tris = nw;
  if (on_device) {
    m.out = tris;
    HIPCHK(c, rm_launch_mc_emit(m, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ROMAP_OK;
  }
  HIPALLOC(c, grow(&c->d_mtris, &c->cap_mtris, (size_t)nw * 9));
  m.out = c->d_mtris;
  HIPCHK(c, rm_launch_mc_emit(m, c->stream));
  HIPCHK(c, hipMemcpyAsync(tris, c->d_mtris, (size_t)nw * 9 * sizeof(float), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ROMAP_OK;
}

romap_status romap_marching_cubes(romap_ctx* c, const float* grid, int32_t res, float iso,
                                  const float lo[3], const float hi[3], float* tris,
                                  int64_t max_tris, int64_t* n_tris, int32_t on_device) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (res < 1 || res > RM_MC_MAX_RES) return fail(c, ROMAP_E_INVALID_ARG, "res must be 1..160");
  if (!grid || !lo || !hi || max_tris < 0) return fail(c, ROMAP_E_INVALID_ARG, "bad buffers");
  romap_status s = mc_setup(c, res);
  if (s != ROMAP_OK) return s;
  const size_t ng = (size_t)(res + 1) * (res + 1) * (res + 1);
  MeshArgs m{};
  if (on_device) {
    m.grid = grid;
  } else {
    HIPCHK(c, hipMemcpyAsync(c->d_mgrid, grid, ng * sizeof(float), hipMemcpyHostToDevice, c->stream));
    m.grid = c->d_mgrid;
  }
  m.res = res;
  m.iso = iso;
  for (int a = 0; a < 3; ++a) {
    m.lo[a] = lo[a];
    m.hi[a] = hi[a];
  }
  return mc_run(c, m, tris, max_tris, n_tris, on_device);
}

romap_status romap_extract_mesh(romap_ctx* c, int32_t id, int32_t res, float iso,
                                int32_t world_frame, float* tris, int64_t max_tris,
                                int64_t* n_tris, int32_t on_device) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (res < 1 || res > RM_MC_MAX_RES) return fail(c, ROMAP_E_INVALID_ARG, "res must be 1..160");
  if (max_tris < 0) return fail(c, ROMAP_E_INVALID_ARG, "bad buffers");
  s = mc_setup(c, res);
  if (s != ROMAP_OK) return s;
  const HostObj& o = c->objs[id];
  HIPCHK(c, rm_launch_density_grid(c->d_objs, id, c->cfg.mlp_layers, res, c->d_mgrid, c->stream));
  MeshArgs m{};
  m.grid = c->d_mgrid;
  m.res = res;
  m.iso = iso;
  for (int a = 0; a < 3; ++a) {
    m.lo[a] = -o.box.half[a];
    m.hi[a] = o.box.half[a];
  }
  if (world_frame) {  // box pose: R = Rz(yaw) in FP64, rounded once
    const double cy = std::cos((double)o.box.yaw), sy = std::sin((double)o.box.yaw);
    const double R[9] = {cy, -sy, 0.0, sy, cy, 0.0, 0.0, 0.0, 1.0};
    m.world = 1;
    for (int k = 0; k < 9; ++k) m.R[k] = (float)R[k];
    for (int a = 0; a < 3; ++a) m.t[a] = o.box.t[a];
  }
  return mc_run(c, m, tris, max_tris, n_tris, on_device);
}

romap_status romap_query_density(romap_ctx* c, int32_t id, const float* xyz, int64_t n,
                                 float* sigma, int32_t on_device) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (n < 0 || (n > 0 && (!xyz || !sigma))) return fail(c, ROMAP_E_INVALID_ARG, "bad buffers");
  if (n == 0) return ROMAP_OK;
  if (on_device) {
    HIPCHK(c, rm_launch_query_density(c->d_objs, id, c->cfg.mlp_layers, xyz, n, sigma, c->stream));
    return ROMAP_OK;
  }
  float *dx = nullptr, *ds = nullptr;
  HIPALLOC(c, hipMalloc((void**)&dx, n * 3 * sizeof(float)));
  hipError_t e = hipMalloc((void**)&ds, n * sizeof(float));
  if (e != hipSuccess) {
    hipFree(dx);
    return fail(c, ROMAP_E_OUT_OF_MEMORY, "query buffers: out of memory");
  }
  HIPCHK(c, hipMemcpyAsync(dx, xyz, n * 3 * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, rm_launch_query_density(c->d_objs, id, c->cfg.mlp_layers, dx, n, ds, c->stream));
  HIPCHK(c, hipMemcpyAsync(sigma, ds, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  hipFree(dx);
  hipFree(ds);
  return ROMAP_OK;
}

static float* kind_ptr(const HostObj& o, int kind) {
  switch (kind) {
    case ROMAP_PARAMS: return o.d_block;
    case ROMAP_GRAD: return o.d_block + o.P_alloc;
    case ROMAP_ADAM_M: return o.d_block + 2 * o.P_alloc;
    case ROMAP_ADAM_V: return o.d_block + 3 * o.P_alloc;
    default: return nullptr;
  }
}

romap_status romap_get_params(romap_ctx* c, int32_t id, int32_t kind, float* buf, int64_t n,
                              int64_t* n_required) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  const HostObj& o = c->objs[id];
  float* src = kind_ptr(o, kind);
  if (!src) return fail(c, ROMAP_E_INVALID_ARG, "bad parameter kind");
  if (n_required) *n_required = o.P;
  if (!buf) return ROMAP_OK;
  if (n < o.P) return fail(c, ROMAP_E_INVALID_ARG, "buffer too small");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(buf, src, o.P * sizeof(float), hipMemcpyDeviceToHost));
  return ROMAP_OK;
}

romap_status romap_set_params(romap_ctx* c, int32_t id, int32_t kind, const float* buf, int64_t n) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  const HostObj& o = c->objs[id];
  float* dst = kind_ptr(o, kind);
  if (!dst) return fail(c, ROMAP_E_INVALID_ARG, "bad parameter kind");
  if (!buf || n != o.P) return fail(c, ROMAP_E_INVALID_ARG, "buffer must hold exactly the object's parameter count");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(dst, buf, o.P * sizeof(float), hipMemcpyHostToDevice));
  if (kind == ROMAP_GRAD) c->objs[id].grad_dirty = true;
  return ROMAP_OK;
}

romap_status romap_debug_rays(romap_ctx* c, int32_t id, int32_t n_rays, int32_t* kf_uv,
                              int32_t* cls, float* ray_f, float* positions) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (n_rays <= 0 || n_rays > (1 << 22)) return fail(c, ROMAP_E_INVALID_ARG, "bad ray count");
  if (c->objs[id].kfs.empty()) return fail(c, ROMAP_E_STATE, "object has no keyframe");
  Plan p;
  build_plan(c, {{id, n_rays}}, 8, 256, p);
  s = stage_plans(c, {&p});
  if (s != ROMAP_OK) return s;
  StepArgs a = plan_args(c, p);
  int32_t* d_kfuv = nullptr;
  float* d_pos = nullptr;
  HIPALLOC(c, hipMalloc((void**)&d_kfuv, (size_t)n_rays * 3 * sizeof(int32_t)));
  a.dbg_kfuv = d_kfuv;
  const int NS = c->cfg.samples_per_ray;
  HIPCHK(c, rm_launch_raygen(a, NS, c->stream));
  if (positions) {
    HIPALLOC(c, hipMalloc((void**)&d_pos, (size_t)p.S * 3 * sizeof(float)));
    HIPCHK(c, rm_launch_debug_positions(a, NS, d_pos, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<RayRec> rr(n_rays);
  HIPCHK(c, hipMemcpy(rr.data(), c->d_rays, n_rays * sizeof(RayRec), hipMemcpyDeviceToHost));
  if (kf_uv) HIPCHK(c, hipMemcpy(kf_uv, d_kfuv, (size_t)n_rays * 3 * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (positions) HIPCHK(c, hipMemcpy(positions, d_pos, (size_t)p.S * 3 * sizeof(float), hipMemcpyDeviceToHost));
  hipFree(d_kfuv);
  hipFree(d_pos);
  for (int r = 0; r < n_rays; ++r) {
    const RayRec& R = rr[r];
    if (cls) cls[r] = (R.flags & RM_F_HIT) ? (int)(R.flags & RM_F_CLS) : -1;
    if (ray_f) {
      float* q = ray_f + 16 * (int64_t)r;
      for (int k = 0; k < 3; ++k) {
        q[k] = R.o[k];
        q[3 + k] = R.d[k];
        q[8 + k] = R.tgt[k];
      }
      q[6] = R.tn;
      q[7] = R.delta;
      q[11] = R.D;
      q[12] = q[13] = q[14] = 0.0f;
      q[15] = (R.flags & RM_F_DEPTH) ? 1.0f : 0.0f;
    }
  }
  return ROMAP_OK;
}

romap_status romap_debug_tiles(romap_ctx* c, int32_t rays_per_item, int32_t gather_block) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (rays_per_item != 4 && rays_per_item != 8 && rays_per_item != 16 && rays_per_item != 32)
    return fail(c, ROMAP_E_INVALID_ARG, "rays_per_item must be 4, 8, 16 or 32");
  if (gather_block != 128 && gather_block != 256 && gather_block != 512)
    return fail(c, ROMAP_E_INVALID_ARG, "gather_block must be 128, 256 or 512");
  c->fixed_rpi = rays_per_item;
  c->fixed_blk = gather_block;
  return ROMAP_OK;
}

romap_status romap_debug_mfma_rate(int32_t precision, double* tflops) {
  if (!tflops || (precision != ROMAP_PREC_FP32 && precision != ROMAP_PREC_BF16))
    return ROMAP_E_INVALID_ARG;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return ROMAP_E_HIP;
  const int blocks = 8 * cus;  // eight 4-wave workgroups per CU: eight waves per SIMD
  const int iters = 2048;
  float* out = nullptr;
  if (hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess) return ROMAP_E_OUT_OF_MEMORY;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  romap_status st = ROMAP_E_HIP;
  float ms = 0.0f;
  const int prec = precision == ROMAP_PREC_BF16 ? 1 : 0;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
      rm_launch_mfma_rate(prec, blocks, 64, out, nullptr) == hipSuccess &&  // warm-up
      hipEventRecord(e0, nullptr) == hipSuccess &&
      rm_launch_mfma_rate(prec, blocks, iters, out, nullptr) == hipSuccess &&
      hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
      hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
    *tflops = rm_mfma_rate_flops(prec, blocks, iters) / (ms * 1e-3) / 1e12;
    st = ROMAP_OK;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  return st;
}

romap_status romap_debug_bin_capacity(romap_ctx* c, int32_t slots) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (slots < 0) return fail(c, ROMAP_E_INVALID_ARG, "slots must be >= 0");
  c->debug_bin_cap = slots;
  return ROMAP_OK;
}

romap_status romap_debug_encode(romap_ctx* c, int32_t id, const float* p, int64_t n, uint32_t* idx,
                                float* feat) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (n <= 0 || !p) return fail(c, ROMAP_E_INVALID_ARG, "bad points");
  const int L = c->objs[id].L;
  float *dp = nullptr, *df = nullptr;
  uint32_t* di = nullptr;
  HIPALLOC(c, hipMalloc((void**)&dp, n * 3 * sizeof(float)));
  HIPALLOC(c, hipMalloc((void**)&df, n * L * 2 * sizeof(float)));
  HIPALLOC(c, hipMalloc((void**)&di, n * L * 8 * sizeof(uint32_t)));
  HIPCHK(c, hipMemcpyAsync(dp, p, n * 3 * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, rm_launch_debug_encode(c->d_objs, id, dp, n, di, df, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (idx) HIPCHK(c, hipMemcpy(idx, di, n * L * 8 * sizeof(uint32_t), hipMemcpyDeviceToHost));
  if (feat) HIPCHK(c, hipMemcpy(feat, df, n * L * 2 * sizeof(float), hipMemcpyDeviceToHost));
  hipFree(dp);
  hipFree(df);
  hipFree(di);
  return ROMAP_OK;
}

static romap_status field_common(romap_ctx* c, int32_t id, const float* params_dev,
                                 const float* rays_dev, int32_t n_rays, Plan& p, StepArgs& a) {
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (!rays_dev || !ray_count_ok(n_rays, c->cfg.samples_per_ray))
    return fail(c, ROMAP_E_INVALID_ARG, "bad rays");
  build_plan(c, {{id, n_rays}}, 8, 256, p);
  p.fins.clear();
  s = stage_plans(c, {&p});
  if (s != ROMAP_OK) return s;
  a = plan_args(c, p);
  a.params_override = params_dev;
  const int NS = c->cfg.samples_per_ray, L = c->cfg.n_levels, K1 = K1_of(c->cfg);
  HIPCHK(c, rm_launch_user_rays(a, NS, rays_dev, c->stream));
  HIPCHK(c, rm_launch_encode_fwd(a, NS, 256, c->stream));
  HIPCHK(c, rm_launch_pack(a, K1, c->stream));
  return ROMAP_OK;
}

romap_status romap_field_forward(romap_ctx* c, int32_t id, const float* params_dev,
                                 const float* rays_dev, int32_t n_rays, float* rgb_dev,
                                 float* depth_dev, float* tend_dev) {
  if (!c) return ROMAP_E_INVALID_ARG;
  Plan p;
  StepArgs a;
  romap_status s = field_common(c, id, params_dev, rays_dev, n_rays, p, a);
  if (s != ROMAP_OK) return s;
  a.mode = RM_MODE_FORWARD;
  a.out_rgb = rgb_dev;
  a.out_depth = depth_dev;
  a.out_tend = tend_dev;
  HIPCHK(c, rm_launch_field(a, c->cfg.samples_per_ray, K1_of(c->cfg), c->cfg.precision, c->stream));
  return ROMAP_OK;
}

romap_status romap_field_forward_noalloc(romap_ctx* c, int32_t id, const float* params_dev,
                                         const float* rays_dev, int32_t n_rays, float* rgb_dev,
                                         float* depth_dev, float* tend_dev) {
  if (!c) return ROMAP_E_INVALID_ARG;
  romap_status s = check_object(c, id);
  if (s != ROMAP_OK) return s;
  if (!rays_dev || !ray_count_ok(n_rays, c->cfg.samples_per_ray))
    return fail(c, ROMAP_E_INVALID_ARG, "bad rays");
  if (!c->scratch_dev) return fail(c, ROMAP_E_STATE, "no scratch on this device");
  // the work lists of romap_field_forward (same launch shape, same kernels)
  Plan p;
  build_plan(c, {{id, n_rays}}, 8, 256, p);
  const int NS = c->cfg.samples_per_ray, K1 = K1_of(c->cfg);
  const size_t L = (size_t)c->cfg.n_levels, WP = RM_WPACK_NH(c->cfg.mlp_layers);
  // carve the scratch: tables | bin counters | rays | encodings | packed weights
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t here = at;
    at += align256(bytes);
    return here;
  };
  const size_t o_sobj = take(p.sobj.size() * sizeof(StepObj));
  const size_t o_items = take(p.items.size() * sizeof(Item));
  const size_t o_bpairs = take(p.bpairs.size() * sizeof(BinPair));
  const size_t o_bblocks = take(p.bblocks.size() * sizeof(BinBlock));
  const size_t tab = at;
  const size_t o_count = take((size_t)p.bin_regions * sizeof(int));
  const size_t o_rays = take((size_t)p.n_rays * sizeof(RayRec));
  const size_t o_e = take(L * (size_t)p.S * sizeof(float2));
  const size_t o_w32 = take(WP * sizeof(float));
  const size_t o_w16 = take(WP * sizeof(uint16_t));
  if (at > RM_SCRATCH_BYTES)
    return fail(c, ROMAP_E_INVALID_ARG,
                "noalloc forward needs " + std::to_string(at) + " bytes of scratch, more than its " +
                    std::to_string(RM_SCRATCH_BYTES) + " (fewer rays per call)");
  char* base = c->scratch_dev;
  std::vector<char> h(tab);
  std::memcpy(h.data() + o_sobj, p.sobj.data(), p.sobj.size() * sizeof(StepObj));
  std::memcpy(h.data() + o_items, p.items.data(), p.items.size() * sizeof(Item));
  if (!p.bpairs.empty()) std::memcpy(h.data() + o_bpairs, p.bpairs.data(), p.bpairs.size() * sizeof(BinPair));
  if (!p.bblocks.empty())
    std::memcpy(h.data() + o_bblocks, p.bblocks.data(), p.bblocks.size() * sizeof(BinBlock));
  HIPCHK(c, hipMemcpyAsync(base, h.data(), tab, hipMemcpyHostToDevice, c->stream));
  StepArgs a = base_args(c);
  a.sobj = (const StepObj*)(base + o_sobj);
  a.n_sobj = (int)p.sobj.size();
  a.items = (const Item*)(base + o_items);
  a.n_items = (int)p.items.size();
  a.fins = nullptr;
  a.n_fins = 0;
  a.n_rays = p.n_rays;
  a.S = p.S;
  a.bpairs = (const BinPair*)(base + o_bpairs);
  a.n_bpairs = (int)p.bpairs.size();
  a.bblocks = (const BinBlock*)(base + o_bblocks);
  a.n_bblocks = (int)p.bblocks.size();
  a.bins = nullptr;
  a.n_bins = 0;
  a.bin_count = (int*)(base + o_count);  // cleared by the gather kernel
  a.n_regions = (int)p.bin_regions;
  a.bin_max_R = 0;
  a.rays = (RayRec*)(base + o_rays);
  a.e = (float2*)(base + o_e);
  a.wpack32 = (float*)(base + o_w32);
  a.wpack16 = (uint16_t*)(base + o_w16);
  a.de = nullptr;  // the forward writes no adjoints, records or partial sums
  a.partials = nullptr;
  a.rec_val = nullptr;
  a.params_override = params_dev;
  a.mode = RM_MODE_FORWARD;
  a.out_rgb = rgb_dev;
  a.out_depth = depth_dev;
  a.out_tend = tend_dev;
  HIPCHK(c, rm_launch_user_rays(a, NS, rays_dev, c->stream));
  HIPCHK(c, rm_launch_encode_fwd(a, NS, 256, c->stream));
  HIPCHK(c, rm_launch_pack(a, K1, c->stream));
  HIPCHK(c, rm_launch_field(a, NS, K1, c->cfg.precision, c->stream));
  // the host copy of the tables must outlive the transfer
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ROMAP_OK;
}

romap_status romap_field_backward(romap_ctx* c, int32_t id, const float* params_dev,
                                  const float* rays_dev, int32_t n_rays, const float* d_rgb_dev,
                                  const float* d_depth_dev, const float* d_tend_dev,
                                  float* d_params_dev) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (!d_params_dev) return fail(c, ROMAP_E_INVALID_ARG, "d_params is NULL");
  Plan p;
  StepArgs a;
  romap_status s = field_common(c, id, params_dev, rays_dev, n_rays, p, a);
  if (s != ROMAP_OK) return s;
  const HostObj& o = c->objs[id];
  a.mode = RM_MODE_ADJOINT;
  a.adj_rgb = d_rgb_dev;
  a.adj_depth = d_depth_dev;
  a.adj_tend = d_tend_dev;
  a.grad_override = d_params_dev;
  const int NS = c->cfg.samples_per_ray, L = c->cfg.n_levels;
  HIPCHK(c, rm_launch_fill(d_params_dev, o.P, 0.0f, c->stream));
  HIPCHK(c, rm_launch_field(a, NS, K1_of(c->cfg), c->cfg.precision, c->stream));
  for (const BinGroup& g : p.bgroups) {
    HIPCHK(c, rm_launch_bin_scatter(a, g, NS, c->stream));
    HIPCHK(c, rm_launch_bin_acc(a, g, c->stream));
  }
  HIPCHK(c, rm_launch_reduce(a, c->stream));
  return ROMAP_OK;
}

// ---- checkpoint -------------------------------------------------------------
static const char kMagic[8] = {'R', 'O', 'M', 'A', 'P', 'C', 'K', '2'};

romap_status romap_save(romap_ctx* c, const char* path) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (!path) return fail(c, ROMAP_E_INVALID_ARG, "path is NULL");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(c, ROMAP_E_INVALID_ARG, std::string("cannot open ") + path);
  bool ok = true;
  auto W = [&](const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; };
  W(kMagic, 8);
  W(&c->cfg, sizeof(c->cfg));
  const int32_t nk = (int32_t)c->kfs.size(), no = (int32_t)c->objs.size();
  W(&nk, 4);
  for (auto& k : c->kfs) {
    W(&k.cam, sizeof(k.cam));
    const size_t npix = (size_t)k.cam.width * k.cam.height;
    std::vector<uint8_t> rgb(npix * 3);
    std::vector<int32_t> mask(npix);
    hipMemcpy(rgb.data(), k.d_rgb, npix * 3, hipMemcpyDeviceToHost);
    hipMemcpy(mask.data(), k.d_mask, npix * 4, hipMemcpyDeviceToHost);
    const int32_t hd = k.d_depth ? 1 : 0;
    W(&hd, 4);
    W(rgb.data(), rgb.size());
    W(mask.data(), mask.size() * 4);
    if (hd) {
      std::vector<float> d(npix);
      hipMemcpy(d.data(), k.d_depth, npix * 4, hipMemcpyDeviceToHost);
      W(d.data(), npix * 4);
    }
  }
  W(&no, 4);
  std::vector<ObjState> st(c->objs.size());
  if (no) hipMemcpy(st.data(), c->d_state, no * sizeof(ObjState), hipMemcpyDeviceToHost);
  for (int i = 0; i < no; ++i) {
    const HostObj& o = c->objs[i];
    W(&o.instance, 4);
    W(&o.log2T, 4);
    W(&o.active, 4);
    W(&o.box, sizeof(o.box));
    W(&st[i].step, 4);
    const int32_t hl = o.has_last;
    W(&hl, 4);
    W(o.last_centre, sizeof(o.last_centre));
    const int32_t nref = (int32_t)o.kfs.size();
    W(&nref, 4);
    for (auto& r : o.kfs) {
      const int32_t v[5] = {r.kf, r.x0, r.y0, r.w, r.h};
      W(v, sizeof(v));
    }
    std::vector<float> buf(3 * o.P_alloc);
    hipMemcpy(buf.data(), o.d_block, o.P_alloc * 4, hipMemcpyDeviceToHost);
    hipMemcpy(buf.data() + o.P_alloc, o.d_block + 2 * o.P_alloc, 2 * o.P_alloc * 4, hipMemcpyDeviceToHost);
    W(buf.data(), buf.size() * 4);
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, ROMAP_E_INVALID_ARG, std::string("write failed: ") + path);
  return ROMAP_OK;
}

romap_status romap_load(romap_ctx* c, const char* path) {
  if (!c) return ROMAP_E_INVALID_ARG;
  if (!path) return fail(c, ROMAP_E_INVALID_ARG, "path is NULL");
  if (!c->objs.empty() || !c->kfs.empty()) return fail(c, ROMAP_E_STATE, "load needs an empty context");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, ROMAP_E_INVALID_ARG, std::string("cannot open ") + path);
  bool ok = true;
  auto R = [&](void* p, size_t n) { ok = ok && std::fread(p, 1, n, f) == n; };
  char magic[8];
  R(magic, 8);
  romap_config cfg;
  R(&cfg, sizeof(cfg));
  if (!ok || std::memcmp(magic, kMagic, 8) != 0) {
    std::fclose(f);
    return fail(c, ROMAP_E_INVALID_ARG, "not a checkpoint");
  }
  if (cfg.n_levels != c->cfg.n_levels || cfg.base_res != c->cfg.base_res || cfg.max_res != c->cfg.max_res ||
      cfg.samples_per_ray != c->cfg.samples_per_ray || cfg.mlp_layers != c->cfg.mlp_layers) {
    std::fclose(f);
    return fail(c, ROMAP_E_INVALID_ARG, "checkpoint model config differs from the context");
  }
  c->cfg.seed = cfg.seed;
  int32_t nk = 0;
  R(&nk, 4);
  std::vector<romap_camera> cams(std::max(nk, 0));
  romap_status s = ROMAP_OK;
  // keyframes: re-added without the acceptance rule; object sets are restored below
  std::vector<int> saved_active;
  for (int i = 0; i < nk && ok; ++i) {
    romap_camera cam;
    R(&cam, sizeof(cam));
    int32_t hd = 0;
    R(&hd, 4);
    if (!ok) break;
    s = validate_camera(c, &cam);  // before sizing buffers from it
    if (s != ROMAP_OK) {
      std::fclose(f);
      return s;
    }
    const size_t npix = (size_t)cam.width * cam.height;
    std::vector<uint8_t> rgb(npix * 3);
    std::vector<int32_t> mask(npix);
    std::vector<float> depth;
    R(rgb.data(), rgb.size());
    R(mask.data(), npix * 4);
    if (hd) {
      depth.resize(npix);
      R(depth.data(), npix * 4);
    }
    if (!ok) break;
    s = romap_add_keyframe(c, &cam, rgb.data(), mask.data(), hd ? depth.data() : nullptr, nullptr, nullptr);
    if (s != ROMAP_OK) {
      std::fclose(f);
      return s;
    }
  }
  int32_t no = 0;
  R(&no, 4);
  for (int i = 0; i < no && ok; ++i) {
    int32_t inst, lt, act, step, hl, nref;
    romap_box box;
    double lc[3];
    R(&inst, 4);
    R(&lt, 4);
    R(&act, 4);
    R(&box, sizeof(box));
    R(&step, 4);
    R(&hl, 4);
    R(lc, sizeof(lc));
    R(&nref, 4);
    if (!ok) break;
    int32_t id = -1;
    s = romap_add_object(c, inst, &box, lt, &id);
    if (s != ROMAP_OK) {
      std::fclose(f);
      return s;
    }
    HostObj& o = c->objs[id];
    o.active = act;
    o.has_last = hl;
    std::memcpy(o.last_centre, lc, sizeof(lc));
    for (int k = 0; k < nref && ok; ++k) {
      int32_t v[5];
      R(v, sizeof(v));
      if (!ok || v[0] < 0 || v[0] >= (int)c->kfs.size()) {
        ok = false;
        break;
      }
      // the ray draw reads the keyframe's pixels inside this rectangle
      const int kw = c->kfs[v[0]].cam.width, kh = c->kfs[v[0]].cam.height;
      if (v[1] < 0 || v[2] < 0 || v[3] < 1 || v[4] < 1 || v[3] > kw - v[1] || v[4] > kh - v[2]) {
        std::fclose(f);
        return fail(c, ROMAP_E_INVALID_ARG, "checkpoint: candidate rectangle outside its keyframe");
      }
      KfRef r{};
      r.kf = v[0];
      r.x0 = v[1];
      r.y0 = v[2];
      r.w = v[3];
      r.h = v[4];
      object_frame(c->kfs[v[0]].cam.T_wc, o.box, r.M, r.c);
      r.cand_begin = o.n_cand;
      o.kfs.push_back(r);
      o.n_cand += (int64_t)r.w * r.h;
    }
    std::vector<float> buf(3 * o.P_alloc);
    R(buf.data(), buf.size() * 4);
    if (!ok) break;
    HIPCHK(c, hipMemcpy(o.d_block, buf.data(), o.P_alloc * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(o.d_block + 2 * o.P_alloc, buf.data() + o.P_alloc, 2 * o.P_alloc * 4, hipMemcpyHostToDevice));
    ObjState st{};
    st.step = step;
    st.bc1 = step ? (float)(1.0 - std::pow((double)c->cfg.beta1, (double)step)) : 1.0f;
    st.bc2 = step ? (float)(1.0 - std::pow((double)c->cfg.beta2, (double)step)) : 1.0f;
    HIPCHK(c, hipMemcpy(c->d_state + id, &st, sizeof(st), hipMemcpyHostToDevice));
    s = upload_object(c, id);
    if (s != ROMAP_OK) {
      std::fclose(f);
      return s;
    }
  }
  std::fclose(f);
  if (!ok) return fail(c, ROMAP_E_INVALID_ARG, "truncated checkpoint");
  return ROMAP_OK;
}

}  // extern "C"
