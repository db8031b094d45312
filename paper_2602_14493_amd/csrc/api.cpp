// C ABI of libgmr: argument validation, the device view table, workspace layout, stage
// orchestration on the caller's stream, and the tile-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gmr_common.h"
#include "gmr_launch.h"

using namespace gmr;

// Stages timed by gmr_profile_* (HIP events around each launch group on the call's stream).
enum Stage { kStProject, kStScanEmit, kStSortFv, kStSortPass, kStRanges, kStRasterFwd, kStFill, kStRasterBwd,
             kStFaceBwd, kStGather, kStBuildSmall, kStRasterStep, kNumStages };
static const char* kStageNames[kNumStages] = {"project",     "scan_emit",  "sort_fv_pass", "sort_pass",
                                              "tile_ranges", "raster_fwd", "fill",         "raster_bwd",
                                              "face_bwd",    "vertex_gather", "build_small", "raster_step"};

struct gmr_ctx {
  int device = 0;
  int num_cus = 256;
  void* scratch = nullptr;  // this device's copy of the static workspace of gmr_render_fwd_noalloc
  std::map<std::string, std::pair<gmr_options, float>> tune_cache;
  bool prof = false;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
};

// Workspace of gmr_render_fwd_noalloc: one static device array, of which every GPU the library
// runs on holds its own copy, at its own address, until the process ends.  Host code never passes
// the array's name to a kernel or a copy (on the host it names a stand-in, not device memory): the
// device address is resolved once per device with hipGetSymbolAddress and used from then on.
static __device__ __align__(256) unsigned char scratch[GMR_NOALLOC_WORKSPACE_BYTES];

namespace {

thread_local std::string g_err;

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // per device: the address of `scratch`, or NULL before resolving

gmr_status fail(gmr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define GMR_CHECK_HIP(expr)                                                                     \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(GMR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Plan {
  int32_t nm = 0, nv = 0;
  int64_t v_total = 0, f_total = 0, fv_total = 0, p_total = 0;
  int32_t tiles_total = 0, items_total = 0, sub_x = 0, sub_y = 0;
  int32_t tile_w = 16, tile_h = 16;
  std::vector<ViewDev> views;
  std::vector<int32_t> mfo, mvo, mvs;
  int32_t max_views = 0;  // most views bound to one mesh
  Layout L{};
  size_t table_bytes = 0;
};

bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

gmr_status validate_options(const gmr_options* o) {
  if (!o) return fail(GMR_ERR_INVALID_ARG, "options is NULL");
  if (o->cov_mode < 0 || o->cov_mode > 2) return fail(GMR_ERR_INVALID_ARG, "cov_mode must be 0, 1 or 2");
  if (!(std::isfinite(o->dilation) && o->dilation >= 0.f)) return fail(GMR_ERR_INVALID_ARG, "dilation must be finite and >= 0");
  if (!(o->alpha_min > 0.f && o->alpha_min < 1.f)) return fail(GMR_ERR_INVALID_ARG, "alpha_min must be in (0, 1)");
  if (!(o->alpha_max >= o->alpha_min && o->alpha_max < 1.f)) return fail(GMR_ERR_INVALID_ARG, "alpha_max must be in [alpha_min, 1)");
  if (!(o->t_eps > 0.f && o->t_eps < 1.f)) return fail(GMR_ERR_INVALID_ARG, "t_eps must be in (0, 1)");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(o->bg[i])) return fail(GMR_ERR_INVALID_ARG, "bg must be finite");
  auto tile_ok = [](int32_t t) { return t >= 8 && t <= 64 && t % 8 == 0; };
  if (!tile_ok(o->tile_w) || !tile_ok(o->tile_h)) return fail(GMR_ERR_INVALID_ARG, "tile_w/tile_h must be multiples of 8 in [8, 64]");
  if (o->raster_mode != 0 && o->raster_mode != 1) return fail(GMR_ERR_INVALID_ARG, "raster_mode must be 0 or 1");
  if (o->px_per_lane != 1 && o->px_per_lane != 2 && o->px_per_lane != 4)
    return fail(GMR_ERR_INVALID_ARG, "px_per_lane must be 1, 2 or 4");
  if (o->tile_h % (kSub * o->px_per_lane) != 0) return fail(GMR_ERR_INVALID_ARG, "tile_h must be a multiple of 8*px_per_lane");
  if (o->lane_lists != 0 && o->lane_lists != 1) return fail(GMR_ERR_INVALID_ARG, "lane_lists must be 0 or 1");
  if (o->sh_degree < 0 || o->sh_degree > 3) return fail(GMR_ERR_INVALID_ARG, "sh_degree must be in [0, 3]");
  if (o->composited_lists < 0 || o->composited_lists > kMaxCompositedLists)
    return fail(GMR_ERR_INVALID_ARG, "composited_lists must be in [0, 8190]");
  return GMR_OK;
}

gmr_status make_plan(const gmr_batch* b, const gmr_options* o, bool need_capacity, Plan& p) {
  gmr_status st = validate_options(o);
  if (st != GMR_OK) return st;
  if (!b) return fail(GMR_ERR_INVALID_ARG, "batch is NULL");
  if (b->num_meshes < 1) return fail(GMR_ERR_INVALID_ARG, "num_meshes must be >= 1");
  if (b->num_views < 1) return fail(GMR_ERR_INVALID_ARG, "num_views must be >= 1");
  if (!b->vert_offsets_host || !b->face_offsets_host || !b->view_mesh_host || !b->cams_host)
    return fail(GMR_ERR_INVALID_ARG, "batch arrays must not be NULL");
  p.nm = b->num_meshes;
  p.nv = b->num_views;
  const int64_t* vo = b->vert_offsets_host;
  const int64_t* fo = b->face_offsets_host;
  if (vo[0] != 0 || fo[0] != 0) return fail(GMR_ERR_INVALID_ARG, "vert_offsets[0] and face_offsets[0] must be 0");
  for (int m = 0; m < p.nm; ++m)
    if (vo[m + 1] < vo[m] || fo[m + 1] < fo[m]) return fail(GMR_ERR_INVALID_ARG, "offsets must be non-decreasing");
  p.v_total = vo[p.nm];
  p.f_total = fo[p.nm];
  if (p.v_total >= (1ll << 31) || p.f_total >= (1ll << 31)) return fail(GMR_ERR_INVALID_ARG, "too many vertices or faces (>= 2^31)");
  p.tile_w = o->tile_w;
  p.tile_h = o->tile_h;
  p.sub_x = o->tile_w / kSub;
  p.sub_y = o->tile_h / (kSub * o->px_per_lane);
  p.views.assign(p.nv, ViewDev{});
  std::vector<std::vector<int32_t>> per_mesh(p.nm);
  int64_t fv = 0, px = 0, tiles = 0;
  for (int v = 0; v < p.nv; ++v) {
    const int32_t m = b->view_mesh_host[v];
    if (m < 0 || m >= p.nm) return fail(GMR_ERR_INVALID_ARG, "view_mesh out of range");
    const gmr_camera& c = b->cams_host[v];
    if (c.width < 1 || c.height < 1 || c.width > 32767 || c.height > 32767)
      return fail(GMR_ERR_INVALID_ARG, "camera width/height must be in [1, 32767]");
    if (!finite_pos(c.fx) || !finite_pos(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
      return fail(GMR_ERR_INVALID_ARG, "camera intrinsics must be finite with fx, fy > 0");
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(c.R[i])) return fail(GMR_ERR_INVALID_ARG, "camera R must be finite");
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(c.t[i])) return fail(GMR_ERR_INVALID_ARG, "camera t must be finite");
    if (!(c.near_plane > 0.f) || !(c.far_plane > c.near_plane)) return fail(GMR_ERR_INVALID_ARG, "need 0 < near_plane < far_plane");
    ViewDev& V = p.views[v];
    std::memcpy(V.R, c.R, sizeof V.R);
    std::memcpy(V.t, c.t, sizeof V.t);
    V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy;
    V.W = c.width; V.H = c.height;
    V.tiles_x = (c.width + p.tile_w - 1) / p.tile_w;
    V.tiles_y = (c.height + p.tile_h - 1) / p.tile_h;
    V.fv_offset = fv;
    V.pixel_offset = px;
    V.tile_base = (int32_t)tiles;
    V.mesh = m;
    V.face_begin = (int32_t)fo[m];
    V.face_end = (int32_t)fo[m + 1];
    V.znear = c.near_plane;
    V.zfar = c.far_plane;
    fv += fo[m + 1] - fo[m];
    px += (int64_t)c.width * c.height;
    tiles += (int64_t)V.tiles_x * V.tiles_y;
    per_mesh[m].push_back(v);
    if (fv >= (1ll << 31) || px >= (1ll << 31) || tiles * p.sub_x * p.sub_y >= (1ll << 31))
      return fail(GMR_ERR_INVALID_ARG, "batch too large (face-views, pixels or raster items >= 2^31)");
  }
  p.fv_total = fv;
  p.p_total = px;
  p.tiles_total = (int32_t)tiles;
  p.items_total = (int32_t)(tiles * p.sub_x * p.sub_y);
  p.mfo.assign(fo, fo + p.nm + 1);
  p.mvo.assign(p.nm + 1, 0);
  p.mvs.clear();
  for (int m = 0; m < p.nm; ++m) {
    p.mvo[m + 1] = p.mvo[m] + (int32_t)per_mesh[m].size();
    p.max_views = std::max(p.max_views, (int32_t)per_mesh[m].size());
    for (int32_t v : per_mesh[m]) p.mvs.push_back(v);
  }
  p.table_bytes = sizeof(TableHdr) + sizeof(ViewDev) * p.nv + sizeof(int32_t) * (2 * (p.nm + 1) + p.nv);

  // workspace layout
  int64_t cap = o->instance_capacity;
  if (need_capacity && (cap <= 0 || cap >= (1ll << 30)))
    return fail(GMR_ERR_INVALID_ARG, "instance_capacity must be in [1, 2^30)");
  if (cap <= 0) cap = 1;
  Layout& L = p.L;
  L.fv_total = p.fv_total;
  L.faces_total = p.f_total;
  L.pixels_total = p.p_total;
  L.capacity = cap;
  L.tiles_total = p.tiles_total;
  L.items_total = p.items_total;
  // tile digits: ceil(bits / 9) passes of at most 9 bits (512 bins), widths as even as possible
  int tile_bits = 0;
  while ((1ll << tile_bits) < p.tiles_total) ++tile_bits;
  L.tile_bits = tile_bits;
  L.tile_passes = std::max(1, (tile_bits + 8) / 9);
  if (L.tile_passes > kMaxPasses - kTileRow0) return fail(GMR_ERR_INVALID_ARG, "too many tiles");
  for (int j = 0, sh = 0; j < L.tile_passes; ++j) {
    const int wbits = (tile_bits - sh + (L.tile_passes - j) - 1) / (L.tile_passes - j);
    L.tile_shift[j] = sh;
    L.tile_mask[j] = (int32_t)((1u << wbits) - 1u);
    sh += wbits;
  }
  L.scan_items = scan_items_for(p.fv_total);
  const int64_t scan_tile = (int64_t)kScanBlock * L.scan_items;
  L.scan_blocks = (int32_t)((p.fv_total + scan_tile - 1) / scan_tile);
  L.sort_items_fv = sort_items_for(p.fv_total);
  L.sort_items_inst = sort_items_for(cap);
  const int64_t part_fv = (int64_t)kSortBlock * L.sort_items_fv, part_inst = (int64_t)kSortBlock * L.sort_items_inst;
  L.parts_fv = (int32_t)((p.fv_total + part_fv - 1) / part_fv);
  L.parts_inst = (int32_t)((cap + part_inst - 1) / part_inst);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t r = off; off = align_up(off + bytes); return r; };
  L.hdr = take(sizeof(WsHdr));
  L.rec = take((size_t)p.fv_total * kRecF4 * 16);
  L.elA = take((size_t)p.fv_total * 16);
  L.elB = take((size_t)p.fv_total * 16);
  L.bdesc = take((size_t)std::max(L.scan_blocks, 1) * 8);
  L.instA = take((size_t)cap * 8);
  L.instB = take((size_t)cap * 8);
  L.keysF = take((size_t)cap * 4);
  L.valsF = take((size_t)cap * 4);
  L.hist = take((size_t)kHistCopies * kHistWords * 4);
  L.descF0 = take((size_t)std::max(L.parts_fv, 1) * 256 * 4);
  L.descF1 = take((size_t)std::max(L.parts_fv, 1) * 256 * 4);
  L.descI0 = take((size_t)L.parts_inst * 512 * 4);
  L.descI1 = take((size_t)L.parts_inst * 512 * 4);
  L.ranges = take((size_t)p.tiles_total * 8);
  L.dfv = take((size_t)p.fv_total * 32);
  L.fgrad = take((size_t)p.f_total * 48);
  L.fsh = take(o->sh_degree > 0 ? (size_t)p.f_total * 12 * (o->sh_degree + 1) * (o->sh_degree + 1) : 0);
  L.statF = take((size_t)std::max(p.items_total, 1) * 8);
  L.statB = take((size_t)std::max(p.items_total, 1) * 16);
  L.statR = take((size_t)kLossReduceBlocks * 16);
  L.total = off;
  return GMR_OK;
}

// The saved buffer: per pixel T_final and the list position after its last composited Gaussian;
// per raster item the block's composited list: a count word, then 16-bit positions.
uint32_t blk_words(const gmr_options* o) {
  return o->composited_lists > 0 ? 1u + ((uint32_t)o->composited_lists + 1u) / 2u : 0u;
}
size_t saved_size(const Plan& p, const gmr_options* o) {
  return (size_t)p.p_total * 8 + (size_t)p.items_total * blk_words(o) * 4;
}

// Raster-block masks in the instance keys: above the tile-id bits, where the tile's blocks fit.
int32_t bm_shift1_of(const Plan& p) {
  int tile_bits = 0;
  while ((1ll << tile_bits) < p.tiles_total) ++tile_bits;
  const int spt = p.sub_x * p.sub_y;
  return (tile_bits <= 26 && spt <= 32 - tile_bits) ? tile_bits + 1 : 0;
}

// The tile-id bits of a sorted key.
uint32_t key_tile_mask(const Plan& p) {
  const int32_t b1 = bm_shift1_of(p);
  return b1 > 0 ? (uint32_t)((1ull << (b1 - 1)) - 1ull) : 0xffffffffu;
}

void write_table(const Plan& p, void* dst) {
  char* base = static_cast<char*>(dst);
  TableHdr h{};
  h.num_views = p.nv;
  h.num_meshes = p.nm;
  h.tile_w = p.tile_w;
  h.tile_h = p.tile_h;
  h.tiles_total = p.tiles_total;
  h.sub_x = p.sub_x;
  h.sub_y = p.sub_y;
  h.items_total = p.items_total;
  h.fv_total = p.fv_total;
  h.pixels_total = p.p_total;
  h.faces_total = p.f_total;
  h.bm_shift1 = bm_shift1_of(p);
  h.views_off = sizeof(TableHdr);
  h.mesh_face_off = h.views_off + (int32_t)(sizeof(ViewDev) * p.nv);
  h.mesh_view_off = h.mesh_face_off + (int32_t)(sizeof(int32_t) * (p.nm + 1));
  h.mesh_views_off = h.mesh_view_off + (int32_t)(sizeof(int32_t) * (p.nm + 1));
  std::memcpy(base, &h, sizeof h);
  std::memcpy(base + h.views_off, p.views.data(), sizeof(ViewDev) * p.nv);
  std::memcpy(base + h.mesh_face_off, p.mfo.data(), sizeof(int32_t) * (p.nm + 1));
  std::memcpy(base + h.mesh_view_off, p.mvo.data(), sizeof(int32_t) * (p.nm + 1));
  std::memcpy(base + h.mesh_views_off, p.mvs.data(), sizeof(int32_t) * p.nv);
}

KOpts kopts(const gmr_options* o) {
  KOpts k;
  k.cov_mode = o->cov_mode;
  k.dilation = o->dilation;
  k.alpha_min = o->alpha_min;
  k.alpha_max = o->alpha_max;
  k.t_eps = o->t_eps;
  k.bg0 = o->bg[0];
  k.bg1 = o->bg[1];
  k.bg2 = o->bg[2];
  k.sh_degree = o->sh_degree;
  k.blk_words = blk_words(o);
  k.blk_cap = (uint32_t)o->composited_lists;
  return k;
}

struct WsPtrs {
  WsHdr* hdr;
  float4* rec;
  uint4* elA;
  uint4* elB;
  uint64_t* bdesc;
  uint2* instA;
  uint2* instB;
  uint32_t* keysF;
  uint32_t* valsF;
  uint32_t* hist;
  uint32_t* descF0;
  uint32_t* descF1;
  uint32_t* descI0;
  uint32_t* descI1;
  uint32_t* ranges;
  float* dfv;
  float4* fgrad;
  float* fsh;
  unsigned long long* statF;
  float4* statB;
  unsigned long long* statR;
  uint32_t* sorted_vals;
};

WsPtrs ws_ptrs(const Layout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  WsPtrs w;
  w.hdr = reinterpret_cast<WsHdr*>(b + L.hdr);
  w.rec = reinterpret_cast<float4*>(b + L.rec);
  w.elA = reinterpret_cast<uint4*>(b + L.elA);
  w.elB = reinterpret_cast<uint4*>(b + L.elB);
  w.bdesc = reinterpret_cast<uint64_t*>(b + L.bdesc);
  w.instA = reinterpret_cast<uint2*>(b + L.instA);
  w.instB = reinterpret_cast<uint2*>(b + L.instB);
  w.keysF = reinterpret_cast<uint32_t*>(b + L.keysF);
  w.valsF = reinterpret_cast<uint32_t*>(b + L.valsF);
  w.hist = reinterpret_cast<uint32_t*>(b + L.hist);
  w.descF0 = reinterpret_cast<uint32_t*>(b + L.descF0);
  w.descF1 = reinterpret_cast<uint32_t*>(b + L.descF1);
  w.descI0 = reinterpret_cast<uint32_t*>(b + L.descI0);
  w.descI1 = reinterpret_cast<uint32_t*>(b + L.descI1);
  w.ranges = reinterpret_cast<uint32_t*>(b + L.ranges);
  w.dfv = reinterpret_cast<float*>(b + L.dfv);
  w.fgrad = reinterpret_cast<float4*>(b + L.fgrad);
  w.fsh = reinterpret_cast<float*>(b + L.fsh);
  w.statF = reinterpret_cast<unsigned long long*>(b + L.statF);
  w.statB = reinterpret_cast<float4*>(b + L.statB);
  w.statR = reinterpret_cast<unsigned long long*>(b + L.statR);
  w.sorted_vals = w.valsF;
  return w;
}

int hist_blocks(const gmr_ctx* h) { return std::max(1, h->num_cus) * 4; }

// Records a HIP event pair around the enclosed launches when profiling is on.
struct StageTimer {
  gmr_ctx* h;
  hipStream_t s;
  gmr_ctx::Rec r;
  bool on;
  StageTimer(gmr_ctx* h_, hipStream_t s_, int stage) : h(h_), s(s_), on(h_ && h_->prof) {
    r.stage = stage;
    if (on) {
      on = hipEventCreate(&r.a) == hipSuccess && hipEventCreate(&r.b) == hipSuccess;
      if (on) (void)hipEventRecord(r.a, s);
    }
  }
  ~StageTimer() {
    if (on) {
      (void)hipEventRecord(r.b, s);
      h->recs.push_back(r);
    }
  }
};

// Conversion + projection + binning + sort (+ optionally zeroing the face-view gradients).
void build_lists(gmr_ctx* h, const Plan& p, const gmr_options* o, const void* table, const float* verts,
                 const int32_t* faces, const float* colors, const WsPtrs& w, bool zero_dfv, hipStream_t s,
                 bool timed = true, bool bwd_follows = false) {
  gmr_ctx* const th = timed ? h : nullptr;  // stage timing records events; untimed calls create none
  const KOpts ko = kopts(o);
  const Layout& L = p.L;
  if (small_build_fits(p.fv_total, p.tiles_total, L.capacity, o->sh_degree)) {  // one launch builds it all
    StageTimer t(th, s, kStBuildSmall);
    const StatsInfo si{(uint32_t)p.items_total, (unsigned long long)L.statF, (unsigned long long)L.statB,
                       bwd_follows ? 1u : 0u};
    launch_build_small(table, verts, faces, colors, ko, w.rec, w.elA, w.hdr,
                       zero_dfv ? reinterpret_cast<float4*>(w.dfv) : nullptr, w.ranges, 2 * p.tiles_total, w.keysF,
                       w.valsF, (uint32_t)L.capacity, si, s);
    return;
  }
  const uint32_t fv_words = (uint32_t)std::max(L.parts_fv, 1) * 256u;
  const uint32_t inst_words = (uint32_t)L.parts_inst * 512u;
  {
    StageTimer t(th, s, kStProject);
    const StatsInfo si{(uint32_t)p.items_total, (unsigned long long)L.statF, (unsigned long long)L.statB,
                       bwd_follows ? 1u : 0u};
    launch_project(table, p.f_total, verts, faces, colors, ko, w.rec, w.elA, w.hist,
                   zero_dfv ? reinterpret_cast<float4*>(w.dfv) : nullptr, w.hdr, w.descF0, fv_words, w.ranges,
                   2 * p.tiles_total, w.bdesc, L.scan_blocks, (uint32_t)L.capacity, si, p.max_views, s);
  }
  // depth digits on the face-view elements: 4 passes, A -> B -> A -> B -> A
  for (int pass = 0; pass < kDepthPasses; ++pass) {
    StageTimer t(th, s, kStSortFv);
    const bool odd = pass & 1;
    launch_sort_fv_pass(odd ? w.elB : w.elA, odd ? w.elA : w.elB, (uint32_t)p.fv_total, w.hist + pass * kHistStride,
                        odd ? w.descF1 : w.descF0, odd ? w.descF0 : w.descF1, fv_words, &w.hdr->part_ctr[pass], pass,
                        w.hdr, L.sort_items_fv, s);
  }
  TilePasses tp;
  tp.n = L.tile_passes;
  for (int j = 0; j < kMaxPasses - kTileRow0; ++j) {
    tp.shift[j] = j < tp.n ? L.tile_shift[j] : 0;
    tp.mask[j] = j < tp.n ? (uint32_t)L.tile_mask[j] : 0u;
  }
  {
    StageTimer t(th, s, kStScanEmit);
    launch_bin(table, w.elA, w.elB, p.fv_total, L.scan_items, w.bdesc, L.scan_blocks, w.hdr, (uint32_t)L.capacity,
               w.instA, w.hist, tp, w.descI0, inst_words, s);
  }
  // tile digits on the instances: A -> B -> A ..., the last pass writes keysF / valsF
  for (int j = 0; j < tp.n; ++j) {
    StageTimer t(th, s, kStSortPass);
    const bool odd = j & 1, last = j + 1 == tp.n;
    launch_sort_inst_pass(odd ? w.instB : w.instA, odd ? w.instA : w.instB, last ? w.keysF : nullptr,
                          last ? w.valsF : nullptr, &w.hdr->count, (uint32_t)L.capacity,
                          w.hist + (kTileRow0 + j) * kHistStride, odd ? w.descI1 : w.descI0, odd ? w.descI0 : w.descI1,
                          last ? 0u : inst_words, &w.hdr->part_ctr[kTileRow0 + j], tp.shift[j], tp.mask[j],
                          L.sort_items_inst, s);
  }
  {
    StageTimer t(th, s, kStRanges);
    launch_tile_ranges(w.keysF, key_tile_mask(p), w.hdr, w.ranges, hist_blocks(h), s);
  }
}

// Persistent schedule: 4 resident workgroups (16 wavefronts) per CU, a multiple of the 8 XCDs.
int persistent_blocks(const gmr_ctx* h, const gmr_options* o) { return o->raster_mode == 1 ? h->num_cus * 4 : 0; }

gmr_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GMR_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return GMR_OK;
}

gmr_status common_checks(gmr_handle h, const void* table, const void* ws, size_t ws_bytes, const Plan& p) {
  if (!h) return fail(GMR_ERR_INVALID_ARG, "handle is NULL");
  if (!table) return fail(GMR_ERR_INVALID_ARG, "table_dev is NULL");
  if (!ws) return fail(GMR_ERR_INVALID_ARG, "ws_dev is NULL");
  if (ws_bytes < p.L.total) return fail(GMR_ERR_WORKSPACE, "workspace smaller than gmr_workspace_size");
  return GMR_OK;
}

// The backward after the compositing adjoint: face-view sums -> face gradients -> vertex gradients
// (with the fused loss's fixed-order sum when red is given).
void bwd_tail(gmr_ctx* h, const Plan& p, const gmr_options* opt, const void* table, const float* verts,
              const int32_t* faces, const float* colors, const WsPtrs& w, const int32_t* adj_off,
              const int32_t* adj_ent, float* d_verts, float* d_colors, const LossRed* red, hipStream_t s) {
  {
    StageTimer t(h, s, kStFaceBwd);
    launch_face_bwd(table, p.f_total, verts, faces, colors, kopts(opt), reinterpret_cast<const float4*>(w.dfv), w.fgrad,
                    w.fsh, p.max_views, s);
  }
  {
    StageTimer t(h, s, kStGather);
    launch_vertex_gather(adj_off, adj_ent, reinterpret_cast<const float*>(w.fgrad), w.fsh, opt->sh_degree, p.v_total,
                         d_verts, d_colors, red, s);
  }
}

gmr_status bwd_impl(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table, const float* verts,
                    const int32_t* faces, const float* colors, const float* d_rgb, const float* d_alpha, const float* rgb,
                    const float* target, float loss_weight, const float* mask, float sil_weight, const void* saved,
                    const int32_t* adj_off, const int32_t* adj_ent, int32_t recompute, float* d_verts, float* d_colors,
                    float* loss_dev, int n_losses, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  gmr_status st = make_plan(batch, opt, true, p);
  if (st != GMR_OK) return st;
  st = common_checks(h, table, ws, ws_bytes, p);
  if (st != GMR_OK) return st;
  if (!verts || !faces || !colors || !saved || !adj_off || !adj_ent || !d_verts || !d_colors)
    return fail(GMR_ERR_INVALID_ARG, "a required device pointer is NULL");
  if (target ? !rgb : !d_rgb) return fail(GMR_ERR_INVALID_ARG, "need d_rgb, or rgb and target for the L2 form");
  if (recompute != 0 && recompute != 1) return fail(GMR_ERR_INVALID_ARG, "recompute_lists must be 0 or 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const WsPtrs w = ws_ptrs(p.L, ws);
  const KOpts ko = kopts(opt);
  if (recompute) build_lists(h, p, opt, table, verts, faces, colors, w, true, s);
  {
    StageTimer t(h, s, kStFill);
    launch_bwd_prologue(w.hdr, w.dfv, recompute ? 0 : p.fv_total * 8, s);
  }
  const float* saved_T = static_cast<const float*>(saved);
  const uint32_t* saved_n = reinterpret_cast<const uint32_t*>(saved_T + p.p_total);
  const uint32_t* saved_blk = blk_words(opt) ? saved_n + p.p_total : nullptr;
  const double n3 = 3.0 * (double)p.p_total;
  {
    StageTimer t(h, s, kStRasterBwd);
    launch_raster_bwd(table, p.items_total, persistent_blocks(h, opt), opt->px_per_lane, w.ranges, w.sorted_vals,
                      w.keysF, w.rec, ko, saved_T, saved_n, saved_blk, d_rgb, d_alpha, rgb, target, (float)(2.0 * loss_weight / n3), (float)(loss_weight / n3),
                      mask, (float)(sil_weight / (double)p.p_total), w.dfv, w.statB, s);
  }
  // fused loss: fixed-order sum of the per-item slots into the header (and loss_dev), carried by
  // the vertex gather's first blocks
  const LossRed red{w.statB, p.items_total, w.statR, w.hdr, loss_dev, n_losses, 0};
  bwd_tail(h, p, opt, table, verts, faces, colors, w, adj_off, adj_ent, d_verts, d_colors, target ? &red : nullptr, s);
  return check_launch();
}

// Regulariser scratch: a float4 per edge and per vertex, then a double per 256-edge and per
// 256-vertex block (the loss partials).
size_t reg_scratch_bytes(int64_t nv, int64_t ne) {
  return (size_t)(ne + nv) * 16 + (size_t)((ne + 255) / 256 + (nv + 255) / 256) * 8;
}

// Unique undirected edges of a triangle list as (i << 32 | j), i < j, ascending.
gmr_status unique_edges(const int32_t* faces, int64_t nf, int64_t nv, std::vector<uint64_t>& keys) {
  keys.clear();
  keys.reserve((size_t)(3 * nf));
  for (int64_t f = 0; f < nf; ++f)
    for (int c = 0; c < 3; ++c) {
      const int32_t a = faces[3 * f + c], b = faces[3 * f + (c + 1) % 3];
      if (a < 0 || a >= nv || b < 0 || b >= nv) return fail(GMR_ERR_INVALID_ARG, "face index out of range");
      if (a == b) continue;
      const uint64_t lo = (uint64_t)std::min(a, b), hi = (uint64_t)std::max(a, b);
      keys.push_back(lo << 32 | hi);
    }
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  return GMR_OK;
}

// The caller's options with only the fields the autotuner chooses taken from `t` (everything else,
// the colour model included, stays the caller's).
gmr_options with_tuned(const gmr_options& base, const gmr_options& t) {
  gmr_options o = base;
  o.tile_w = t.tile_w;
  o.tile_h = t.tile_h;
  o.px_per_lane = t.px_per_lane;
  o.raster_mode = t.raster_mode;
  o.lane_lists = t.lane_lists;
  o.instance_capacity = t.instance_capacity;
  return o;
}

std::string tune_key(const Plan& p, const gmr_options* o) {
  std::string k = std::to_string(p.nv) + ":" + std::to_string(p.f_total) + ":" + std::to_string(o->cov_mode) + ":" +
                  std::to_string(o->sh_degree);
  for (const ViewDev& v : p.views) k += ":" + std::to_string(v.W) + "x" + std::to_string(v.H);
  return k;
}

}  // namespace

// ================================================================================================
extern "C" {

gmr_options gmr_default_options(void) {
  gmr_options o;
  std::memset(&o, 0, sizeof o);
  o.cov_mode = 0;
  o.dilation = 0.3f;
  o.alpha_min = 1.0f / 255.0f;
  o.alpha_max = 0.99f;
  o.t_eps = 1e-4f;
  o.bg[0] = o.bg[1] = o.bg[2] = 0.f;
  o.tile_w = 16;
  o.tile_h = 16;
  o.raster_mode = 0;
  o.px_per_lane = 1;
  o.lane_lists = 1;
  o.sh_degree = 0;
  o.composited_lists = 2046;
  o.instance_capacity = 0;
  return o;
}

const char* gmr_status_string(gmr_status s) {
  switch (s) {
    case GMR_OK: return "ok";
    case GMR_ERR_INVALID_ARG: return "invalid argument";
    case GMR_ERR_WORKSPACE: return "workspace too small";
    case GMR_ERR_CAPACITY: return "instance capacity exceeded";
    case GMR_ERR_UNSUPPORTED: return "unsupported";
    case GMR_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* gmr_last_error(void) { return g_err.c_str(); }

gmr_status gmr_create(gmr_handle* out, int device) {
  if (!out) return fail(GMR_ERR_INVALID_ARG, "out is NULL");
  int n = 0;
  GMR_CHECK_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(GMR_ERR_INVALID_ARG, "device out of range");
  hipDeviceProp_t prop;
  GMR_CHECK_HIP(hipGetDeviceProperties(&prop, device));
  // the device address of the static workspace, resolved once per device with that device current
  void* sp = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() < n) g_scratch_dev.resize(n, nullptr);
    if (!g_scratch_dev[device]) {
      int prev = 0;
      GMR_CHECK_HIP(hipGetDevice(&prev));
      GMR_CHECK_HIP(hipSetDevice(device));
      const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
      (void)hipSetDevice(prev);
      if (e != hipSuccess || !sp)
        return fail(GMR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_scratch_dev[device] = sp;
    }
    sp = g_scratch_dev[device];
  }
  gmr_ctx* c = new gmr_ctx;
  c->device = device;
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->scratch = sp;
  *out = c;
  return GMR_OK;
}

gmr_status gmr_destroy(gmr_handle h) {
  delete h;
  return GMR_OK;
}

gmr_status gmr_view_table_size(const gmr_batch* batch, const gmr_options* opt, size_t* bytes) {
  if (!bytes) return fail(GMR_ERR_INVALID_ARG, "bytes is NULL");
  Plan p;
  gmr_status st = make_plan(batch, opt, false, p);
  if (st != GMR_OK) return st;
  *bytes = p.table_bytes;
  return GMR_OK;
}

gmr_status gmr_view_table_fill(const gmr_batch* batch, const gmr_options* opt, void* host_dst, size_t bytes) {
  if (!host_dst) return fail(GMR_ERR_INVALID_ARG, "host_dst is NULL");
  Plan p;
  gmr_status st = make_plan(batch, opt, false, p);
  if (st != GMR_OK) return st;
  if (bytes < p.table_bytes) return fail(GMR_ERR_INVALID_ARG, "view table buffer too small");
  write_table(p, host_dst);
  return GMR_OK;
}

gmr_status gmr_workspace_size(const gmr_batch* batch, const gmr_options* opt, size_t* ws_bytes, size_t* saved_bytes) {
  if (!ws_bytes || !saved_bytes) return fail(GMR_ERR_INVALID_ARG, "output pointer is NULL");
  Plan p;
  gmr_status st = make_plan(batch, opt, true, p);
  if (st != GMR_OK) return st;
  *ws_bytes = p.L.total;
  *saved_bytes = saved_size(p, opt);
  return GMR_OK;
}

gmr_status gmr_build_adjacency(const int32_t* faces, int64_t nf, int64_t nv, int32_t* off, int32_t* ent) {
  if (!faces || !off || !ent || nf < 0 || nv < 0) return fail(GMR_ERR_INVALID_ARG, "bad adjacency arguments");
  if (3 * nf >= (1ll << 31)) return fail(GMR_ERR_INVALID_ARG, "too many faces");
  std::vector<int32_t> cnt(nv + 1, 0);
  for (int64_t i = 0; i < 3 * nf; ++i) {
    const int32_t v = faces[i];
    if (v < 0 || v >= nv) return fail(GMR_ERR_INVALID_ARG, "face index out of range");
    cnt[v + 1]++;
  }
  off[0] = 0;
  for (int64_t v = 0; v < nv; ++v) off[v + 1] = off[v] + cnt[v + 1];
  std::vector<int32_t> cur(off, off + nv);
  for (int64_t i = 0; i < 3 * nf; ++i) ent[cur[faces[i]]++] = (int32_t)i;  // i = face * 3 + corner, ascending
  return GMR_OK;
}

namespace {
// The forward's launches into workspace ws (validated by the caller).
void fwd_impl(gmr_ctx* h, const Plan& p, const gmr_options* opt, const void* table, const float* verts,
              const int32_t* faces, const float* colors, float* out_rgb, float* out_alpha, void* saved, void* ws,
              bool timed, hipStream_t s) {
  const WsPtrs w = ws_ptrs(p.L, ws);
  build_lists(h, p, opt, table, verts, faces, colors, w, false, s, timed);
  float* saved_T = static_cast<float*>(saved);
  uint32_t* saved_n = reinterpret_cast<uint32_t*>(saved_T + p.p_total);
  uint32_t* saved_blk = blk_words(opt) ? saved_n + p.p_total : nullptr;
  {
    StageTimer t(timed ? h : nullptr, s, kStRasterFwd);
    launch_raster_fwd(table, p.items_total, persistent_blocks(h, opt), opt->px_per_lane, opt->lane_lists != 0, w.ranges,
                      w.sorted_vals, w.keysF, w.rec, kopts(opt),
                      out_rgb, out_alpha, saved_T, saved_n, saved_blk, w.statF, s);
  }
}
}  // namespace

gmr_status gmr_render_fwd(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                          const float* verts, const int32_t* faces, const float* colors, float* out_rgb, float* out_alpha,
                          void* saved, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  gmr_status st = make_plan(batch, opt, true, p);
  if (st != GMR_OK) return st;
  st = common_checks(h, table, ws, ws_bytes, p);
  if (st != GMR_OK) return st;
  if (!verts || !faces || !colors || !out_rgb || !saved) return fail(GMR_ERR_INVALID_ARG, "a required device pointer is NULL");
  fwd_impl(h, p, opt, table, verts, faces, colors, out_rgb, out_alpha, saved, ws, true, static_cast<hipStream_t>(stream));
  return check_launch();
}

gmr_status gmr_render_fwd_noalloc(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                                  const float* verts, const int32_t* faces, const float* colors, float* out_rgb,
                                  float* out_alpha, void* saved, uint32_t* counters, void* stream) {
  Plan p;
  gmr_status st = make_plan(batch, opt, true, p);
  if (st != GMR_OK) return st;
  if (!h) return fail(GMR_ERR_INVALID_ARG, "handle is NULL");
  if (!h->scratch) return fail(GMR_ERR_HIP, "the static workspace of this device was not resolved");
  if (p.L.total > GMR_NOALLOC_WORKSPACE_BYTES)
    return fail(GMR_ERR_WORKSPACE, "this batch needs " + std::to_string(p.L.total) +
                                       " workspace bytes; the static workspace holds " +
                                       std::to_string((size_t)GMR_NOALLOC_WORKSPACE_BYTES) +
                                       " (use gmr_render_fwd with a caller workspace, or a smaller instance_capacity)");
  st = common_checks(h, table, h->scratch, GMR_NOALLOC_WORKSPACE_BYTES, p);
  if (st != GMR_OK) return st;
  if (!verts || !faces || !colors || !out_rgb || !saved) return fail(GMR_ERR_INVALID_ARG, "a required device pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every region the forward reads is written earlier in the same call (its prologue clears the
  // counters, tickets, descriptors, histograms and tile ranges), so the previous call's contents
  // need no clearing here
  fwd_impl(h, p, opt, table, verts, faces, colors, out_rgb, out_alpha, saved, h->scratch, false, s);
  if (counters)  // {instance count, overflow flag}: the first two words of the workspace header
    GMR_CHECK_HIP(hipMemcpyAsync(counters, h->scratch, 2 * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  return check_launch();
}

gmr_status gmr_profile_enable(gmr_handle h, int32_t enable) {
  if (!h) return fail(GMR_ERR_INVALID_ARG, "handle is NULL");
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  h->recs.clear();
  h->prof = enable != 0;
  return GMR_OK;
}

gmr_status gmr_profile_read(gmr_handle h, int32_t max_stages, char* names, float* ms_total, int32_t* launches,
                            int32_t* n_stages) {
  if (!h || !names || !ms_total || !launches || !n_stages || max_stages < kNumStages)
    return fail(GMR_ERR_INVALID_ARG, "bad profile arguments");
  for (int i = 0; i < kNumStages; ++i) {
    std::memset(names + 32 * i, 0, 32);
    std::strncpy(names + 32 * i, kStageNames[i], 31);
    ms_total[i] = 0.f;
    launches[i] = 0;
  }
  for (auto& r : h->recs) {
    GMR_CHECK_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    GMR_CHECK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    ms_total[r.stage] += ms;
    launches[r.stage] += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  h->recs.clear();
  *n_stages = kNumStages;
  return GMR_OK;
}

gmr_status gmr_render_bwd(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                          const float* verts, const int32_t* faces, const float* colors, const float* d_rgb,
                          const float* d_alpha, const void* saved, const int32_t* adj_off, const int32_t* adj_ent,
                          int32_t recompute, float* d_verts, float* d_colors, void* ws, size_t ws_bytes, void* stream) {
  return bwd_impl(h, batch, opt, table, verts, faces, colors, d_rgb, d_alpha, nullptr, nullptr, 0.f, nullptr, 0.f, saved,
                  adj_off, adj_ent, recompute, d_verts, d_colors, nullptr, 0, ws, ws_bytes, stream);
}

gmr_status gmr_render_bwd_l2(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                             const float* verts, const int32_t* faces, const float* colors, const float* rgb,
                             const float* target, float loss_weight, const void* saved, const int32_t* adj_off,
                             const int32_t* adj_ent, int32_t recompute, float* d_verts, float* d_colors, float* loss_dev,
                             void* ws, size_t ws_bytes, void* stream) {
  if (!rgb || !target) return fail(GMR_ERR_INVALID_ARG, "rgb and target must not be NULL");
  if (!std::isfinite(loss_weight)) return fail(GMR_ERR_INVALID_ARG, "loss_weight must be finite");
  return bwd_impl(h, batch, opt, table, verts, faces, colors, nullptr, nullptr, rgb, target, loss_weight, nullptr, 0.f,
                  saved, adj_off, adj_ent, recompute, d_verts, d_colors, loss_dev, 1, ws, ws_bytes, stream);
}

namespace {
// One step's rendering from a single list build (gmr_render_step_l2 / _recon): forward, then the
// fused colour (and, with a mask, silhouette) backward.
gmr_status step_impl(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                     const float* verts, const int32_t* faces, const float* colors, const float* target,
                     float color_weight, const float* mask, float sil_weight, float* out_rgb, float* out_alpha,
                     void* saved, const int32_t* adj_off, const int32_t* adj_ent, float* d_verts, float* d_colors,
                     float* losses_dev, int n_losses, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  gmr_status st = make_plan(batch, opt, true, p);
  if (st != GMR_OK) return st;
  st = common_checks(h, table, ws, ws_bytes, p);
  if (st != GMR_OK) return st;
  if (!verts || !faces || !colors || !target || !out_rgb || !saved || !adj_off || !adj_ent || !d_verts || !d_colors)
    return fail(GMR_ERR_INVALID_ARG, "a required device pointer is NULL");
  if (!std::isfinite(color_weight) || !std::isfinite(sil_weight))
    return fail(GMR_ERR_INVALID_ARG, "loss weights must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const WsPtrs w = ws_ptrs(p.L, ws);
  const KOpts ko = kopts(opt);
  // the projection also clears dfv, and the build's prologue sets up the backward's counters
  build_lists(h, p, opt, table, verts, faces, colors, w, true, s, true, true);
  float* saved_T = static_cast<float*>(saved);
  uint32_t* saved_n = reinterpret_cast<uint32_t*>(saved_T + p.p_total);
  uint32_t* saved_blk = blk_words(opt) ? saved_n + p.p_total : nullptr;
  const double n3 = 3.0 * (double)p.p_total;
  const float gs = (float)(2.0 * color_weight / n3), ls = (float)(color_weight / n3);
  const float ss = (float)(sil_weight / (double)p.p_total);
  if (opt->px_per_lane == 1 && persistent_blocks(h, opt) == 0) {  // one launch composites and differentiates
    StageTimer t(h, s, kStRasterStep);
    launch_raster_step(table, p.items_total, opt->lane_lists != 0, w.ranges, w.sorted_vals, w.keysF, w.rec, ko,
                       out_rgb, out_alpha, saved_T, saved_n, saved_blk, w.statF, target, gs, ls, mask, ss, w.dfv,
                       w.statB, s);
  } else {
    {
      StageTimer t(h, s, kStRasterFwd);
      launch_raster_fwd(table, p.items_total, persistent_blocks(h, opt), opt->px_per_lane, opt->lane_lists != 0,
                        w.ranges, w.sorted_vals, w.keysF, w.rec, ko, out_rgb, out_alpha, saved_T, saved_n, saved_blk,
                        w.statF, s);
    }
    {
      StageTimer t(h, s, kStRasterBwd);
      launch_raster_bwd(table, p.items_total, persistent_blocks(h, opt), opt->px_per_lane, w.ranges, w.sorted_vals,
                        w.keysF, w.rec, ko, saved_T, saved_n, saved_blk, nullptr, nullptr, out_rgb, target, gs, ls, mask,
                        ss, w.dfv,
                        w.statB, s);
    }
  }
  const LossRed red{w.statB, p.items_total, w.statR, w.hdr, losses_dev, n_losses, 0};
  bwd_tail(h, p, opt, table, verts, faces, colors, w, adj_off, adj_ent, d_verts, d_colors, &red, s);
  return check_launch();
}
}  // namespace

gmr_status gmr_render_step_l2(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                              const float* verts, const int32_t* faces, const float* colors, const float* target,
                              float loss_weight, float* out_rgb, float* out_alpha, void* saved, const int32_t* adj_off,
                              const int32_t* adj_ent, float* d_verts, float* d_colors, float* loss_dev, void* ws,
                              size_t ws_bytes, void* stream) {
  return step_impl(h, batch, opt, table, verts, faces, colors, target, loss_weight, nullptr, 0.f, out_rgb, out_alpha,
                   saved, adj_off, adj_ent, d_verts, d_colors, loss_dev, 1, ws, ws_bytes, stream);
}

gmr_status gmr_render_step_recon(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                                 const float* verts, const int32_t* faces, const float* colors, const float* target,
                                 float color_weight, const float* mask, float sil_weight, float* out_rgb,
                                 float* out_alpha, void* saved, const int32_t* adj_off, const int32_t* adj_ent,
                                 float* d_verts, float* d_colors, float* losses_dev, void* ws, size_t ws_bytes,
                                 void* stream) {
  if (!mask) return fail(GMR_ERR_INVALID_ARG, "mask must not be NULL");
  return step_impl(h, batch, opt, table, verts, faces, colors, target, color_weight, mask, sil_weight, out_rgb,
                   out_alpha, saved, adj_off, adj_ent, d_verts, d_colors, losses_dev, 2, ws, ws_bytes, stream);
}

gmr_status gmr_render_bwd_recon(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table,
                                const float* verts, const int32_t* faces, const float* colors, const float* rgb,
                                const float* target, float color_weight, const float* mask, float sil_weight,
                                const void* saved, const int32_t* adj_off, const int32_t* adj_ent, int32_t recompute,
                                float* d_verts, float* d_colors, float* losses_dev, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!rgb || !target || !mask) return fail(GMR_ERR_INVALID_ARG, "rgb, target and mask must not be NULL");
  if (!std::isfinite(color_weight) || !std::isfinite(sil_weight))
    return fail(GMR_ERR_INVALID_ARG, "loss weights must be finite");
  return bwd_impl(h, batch, opt, table, verts, faces, colors, nullptr, nullptr, rgb, target, color_weight, mask,
                  sil_weight, saved, adj_off, adj_ent, recompute, d_verts, d_colors, losses_dev, 2, ws, ws_bytes, stream);
}

gmr_status gmr_mesh_graph_size(const int32_t* faces, int64_t nf, int64_t nv, int64_t* num_edges) {
  if (!faces || !num_edges || nf < 0 || nv < 0) return fail(GMR_ERR_INVALID_ARG, "bad mesh graph arguments");
  std::vector<uint64_t> keys;
  gmr_status st = unique_edges(faces, nf, nv, keys);
  if (st != GMR_OK) return st;
  *num_edges = (int64_t)keys.size();
  return GMR_OK;
}

gmr_status gmr_build_mesh_graph(const int32_t* faces, int64_t nf, int64_t nv, int64_t num_edges, int32_t* edges,
                                int32_t* vedge_off, int32_t* vedge_ent) {
  if (!faces || !edges || !vedge_off || !vedge_ent || nf < 0 || nv < 0) return fail(GMR_ERR_INVALID_ARG, "bad mesh graph arguments");
  std::vector<uint64_t> keys;
  gmr_status st = unique_edges(faces, nf, nv, keys);
  if (st != GMR_OK) return st;
  if ((int64_t)keys.size() != num_edges) return fail(GMR_ERR_INVALID_ARG, "num_edges does not match the mesh");
  if (2 * num_edges >= (1ll << 30)) return fail(GMR_ERR_INVALID_ARG, "too many edges");
  std::vector<int32_t> cnt(nv + 1, 0);
  for (int64_t e = 0; e < num_edges; ++e) {
    edges[2 * e] = (int32_t)(keys[e] >> 32);
    edges[2 * e + 1] = (int32_t)(keys[e] & 0xffffffffu);
    cnt[edges[2 * e] + 1]++;
    cnt[edges[2 * e + 1] + 1]++;
  }
  vedge_off[0] = 0;
  for (int64_t v = 0; v < nv; ++v) vedge_off[v + 1] = vedge_off[v] + cnt[v + 1];
  std::vector<int32_t> cur(vedge_off, vedge_off + nv);
  for (int64_t e = 0; e < num_edges; ++e) {  // ascending edge index per vertex
    vedge_ent[cur[edges[2 * e]]++] = (int32_t)(e << 1);            // side 0: first end
    vedge_ent[cur[edges[2 * e + 1]]++] = (int32_t)((e << 1) | 1);  // side 1: second end
  }
  return GMR_OK;
}

gmr_status gmr_regularizers_scratch_size(int64_t nv, int64_t num_edges, size_t* bytes) {
  if (!bytes || nv < 0 || num_edges < 0) return fail(GMR_ERR_INVALID_ARG, "bad arguments");
  *bytes = reg_scratch_bytes(nv, num_edges);
  return GMR_OK;
}

gmr_status gmr_regularizers(const float* verts, int64_t nv, const int32_t* edges, int64_t num_edges,
                            const int32_t* vedge_off, const int32_t* vedge_ent, float target_length, float edge_weight,
                            float lap_weight, void* scratch, size_t scratch_bytes, float* losses, float* d_verts,
                            void* stream) {
  if (!verts || !edges || !vedge_off || !vedge_ent || !scratch || !losses || !d_verts || nv < 0 || num_edges < 0)
    return fail(GMR_ERR_INVALID_ARG, "bad regularizer arguments");
  if (scratch_bytes < reg_scratch_bytes(nv, num_edges)) return fail(GMR_ERR_WORKSPACE, "regularizer scratch too small");
  if (!std::isfinite(target_length) || !std::isfinite(edge_weight) || !std::isfinite(lap_weight))
    return fail(GMR_ERR_INVALID_ARG, "regularizer parameters must be finite");
  float4* ge = static_cast<float4*>(scratch);
  launch_regularizers(verts, nv, edges, num_edges, vedge_off, vedge_ent, target_length, edge_weight, lap_weight, ge,
                      ge + num_edges, reinterpret_cast<double*>(ge + num_edges + nv), losses, d_verts,
                      static_cast<hipStream_t>(stream));
  return check_launch();
}

gmr_status gmr_vector_adam_step(float* param, const float* grad, float* m, float* v, int64_t nv, float lr, float beta1,
                                float beta2, float eps, int32_t* step, void* stream) {
  if (!param || !grad || !m || !v || !step || nv < 0) return fail(GMR_ERR_INVALID_ARG, "bad VectorAdam arguments");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(GMR_ERR_INVALID_ARG, "bad VectorAdam hyper-parameters");
  launch_vector_adam(param, grad, m, v, nv, lr, beta1, beta2, eps, step, static_cast<hipStream_t>(stream));
  return check_launch();
}

gmr_status gmr_workspace_view(const gmr_batch* batch, const gmr_options* opt, size_t* ranges_off, size_t* vals_off,
                              size_t* rec_off, size_t* keys_off) {
  if (!ranges_off || !vals_off || !rec_off || !keys_off) return fail(GMR_ERR_INVALID_ARG, "output pointer is NULL");
  Plan p;
  gmr_status st = make_plan(batch, opt, true, p);
  if (st != GMR_OK) return st;
  *ranges_off = p.L.ranges;
  *vals_off = p.L.valsF;
  *rec_off = p.L.rec;
  *keys_off = p.L.keysF;
  return GMR_OK;
}

gmr_status gmr_read_counters(const void* ws, size_t ws_bytes, gmr_counters* out, void* stream) {
  if (!ws || !out || ws_bytes < sizeof(WsHdr)) return fail(GMR_ERR_INVALID_ARG, "bad arguments");
  WsHdr hdr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  GMR_CHECK_HIP(hipMemcpyAsync(&hdr, ws, sizeof hdr, hipMemcpyDeviceToHost, s));
  GMR_CHECK_HIP(hipStreamSynchronize(s));
  out->instances = hdr.count;
  out->capacity = hdr.capacity;
  out->overflow = (int32_t)hdr.overflow;
  out->peak_instances = hdr.peak_count;
  out->overflow_any = hdr.peak_count > hdr.capacity ? 1 : 0;
  {  // restart the peak: the next read covers the builds after this one
    const uint32_t zero = 0u;
    GMR_CHECK_HIP(hipMemcpyAsync(static_cast<char*>(const_cast<void*>(ws)) + offsetof(WsHdr, peak_count), &zero,
                                 sizeof zero, hipMemcpyHostToDevice, s));
    GMR_CHECK_HIP(hipStreamSynchronize(s));
  }
  // pair counts: sums of the raster kernels' per-item slots
  out->pairs_fwd = 0;
  out->pairs_bwd = 0;
  const size_t items = hdr.stats_items;
  if (items > 0 && hdr.stats_fwd_off + items * 8 <= ws_bytes && hdr.stats_bwd_off + items * 16 <= ws_bytes) {
    const char* b = static_cast<const char*>(ws);
    std::vector<unsigned long long> f(items);
    GMR_CHECK_HIP(hipMemcpyAsync(f.data(), b + hdr.stats_fwd_off, items * 8, hipMemcpyDeviceToHost, s));
    std::vector<uint32_t> bw;
    if (hdr.bwd_stats) {
      bw.resize(items * 4);
      GMR_CHECK_HIP(hipMemcpyAsync(bw.data(), b + hdr.stats_bwd_off, items * 16, hipMemcpyDeviceToHost, s));
    }
    GMR_CHECK_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < items; ++i) out->pairs_fwd += (int64_t)f[i];
    for (size_t i = 0; i < bw.size(); i += 4) out->pairs_bwd += (int64_t)((uint64_t)bw[i + 2] | ((uint64_t)bw[i + 3] << 32));
  }
  out->loss = hdr.loss;
  out->loss_sil = hdr.loss_sil;
  return GMR_OK;
}

gmr_status gmr_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                         int32_t* step, void* stream) {
  if (!p || !g || !m || !v || !step || n < 0) return fail(GMR_ERR_INVALID_ARG, "bad Adam arguments");
  if (!(b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps > 0.f && std::isfinite(lr)))
    return fail(GMR_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  launch_adam(p, g, m, v, n, lr, b1, b2, eps, step, static_cast<hipStream_t>(stream));
  return check_launch();
}

gmr_status gmr_autotune(gmr_handle h, const gmr_batch* batch, const gmr_options* base, const float* verts,
                        const int32_t* faces, const float* colors, const float* target, const int32_t* adj_off,
                        const int32_t* adj_ent, int32_t iters, int32_t recompute, gmr_options* best_out, float* ms_out,
                        void* stream) {
  if (!h || !best_out || !verts || !faces || !colors || !target || !adj_off || !adj_ent || iters < 1)
    return fail(GMR_ERR_INVALID_ARG, "bad autotune arguments");
  if (recompute != 0 && recompute != 1) return fail(GMR_ERR_INVALID_ARG, "recompute must be 0 or 1");
  Plan p0;
  gmr_options b = *base;
  if (b.instance_capacity <= 0) b.instance_capacity = 1;
  gmr_status st = make_plan(batch, &b, true, p0);
  if (st != GMR_OK) return st;
  const std::string key = tune_key(p0, &b) + ":r" + std::to_string(recompute);
  auto it = h->tune_cache.find(key);
  if (it != h->tune_cache.end()) {
    *best_out = with_tuned(*base, it->second.first);
    if (ms_out) *ms_out = it->second.second;
    return GMR_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // candidates: binning tile, pixels per lane (block shape), raster mode
  struct Cand { int tw, th, px, mode, lanes; };
  std::vector<Cand> cands;
  // 64 x 64 lets a small batch sort its tile ids in one pass (512 tiles: 8 views of 512^2)
  const int shapes[][2] = {{8, 8}, {16, 16}, {32, 16}, {32, 32}, {64, 32}, {64, 64}};
  for (const auto& sh : shapes)
    for (int px : {1, 2, 4})
      if (sh[1] % (kSub * px) == 0)
        for (int mode = 0; mode < 2; ++mode)
          for (int lanes = 0; lanes < 2; ++lanes) cands.push_back({sh[0], sh[1], px, mode, lanes});
  // the search's own scratch, released on every return path
  struct Scratch {
    float *rgb = nullptr, *dv = nullptr, *dc = nullptr;
    void *saved = nullptr, *ws = nullptr, *table = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Scratch() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      for (void* q : {(void*)rgb, (void*)dv, (void*)dc, saved, ws, table})
        if (q) (void)hipFree(q);
    }
  } sc;
  float *&rgb = sc.rgb, *&dv = sc.dv, *&dc = sc.dc;
  void *&saved = sc.saved, *&ws = sc.ws, *&table = sc.table;
  hipEvent_t &e0 = sc.e0, &e1 = sc.e1;
  size_t ws_cap = 0, table_cap = 0, saved_cap = 0;  // grown per candidate (their raster items differ)
  GMR_CHECK_HIP(hipMalloc(&rgb, sizeof(float) * 3 * p0.p_total));
  GMR_CHECK_HIP(hipMalloc(&dv, sizeof(float) * 3 * p0.v_total));
  // colour gradients have the colours' layout: (sh_degree + 1)^2 coefficients per channel
  const size_t n_coef = (size_t)(b.sh_degree + 1) * (b.sh_degree + 1);
  GMR_CHECK_HIP(hipMalloc(&dc, sizeof(float) * 3 * n_coef * p0.v_total));
  GMR_CHECK_HIP(hipEventCreate(&e0));
  GMR_CHECK_HIP(hipEventCreate(&e1));
  gmr_status result = GMR_OK;
  // Times one candidate: forward + fused L2 backward (lists rebuilt in the backward when
  // recompute = 1), iters timed steps after a warm-up step.  On return o.instance_capacity holds
  // the measured count with 25 % headroom.
  auto time_cand = [&](gmr_options& o, float& ms_out_c) -> gmr_status {
    bool tightened = false;
    for (int attempt = 0; attempt < 4; ++attempt) {
      Plan p;
      gmr_status r;
      if ((r = make_plan(batch, &o, true, p)) != GMR_OK) return r;
      if (p.table_bytes > table_cap) {
        if (table) (void)hipFree(table);
        table = nullptr;
        table_cap = p.table_bytes;
        if (hipMalloc(&table, table_cap) != hipSuccess) return fail(GMR_ERR_HIP, "autotune: hipMalloc");
      }
      std::vector<char> tb(p.table_bytes);
      write_table(p, tb.data());
      if (hipMemcpy(table, tb.data(), p.table_bytes, hipMemcpyHostToDevice) != hipSuccess)
        return fail(GMR_ERR_HIP, "autotune: hipMemcpy");
      if (p.L.total > ws_cap) {
        if (ws) (void)hipFree(ws);
        ws = nullptr;
        ws_cap = p.L.total;
        if (hipMalloc(&ws, ws_cap) != hipSuccess) return fail(GMR_ERR_HIP, "autotune: hipMalloc workspace");
      }
      if (saved_size(p, &o) > saved_cap) {
        if (saved) (void)hipFree(saved);
        saved = nullptr;
        saved_cap = saved_size(p, &o);
        if (hipMalloc(&saved, saved_cap) != hipSuccess) return fail(GMR_ERR_HIP, "autotune: hipMalloc saved");
      }
      if ((r = gmr_render_fwd(h, batch, &o, table, verts, faces, colors, rgb, nullptr, saved, ws, ws_cap, s)) != GMR_OK)
        return r;
      gmr_counters c;
      if ((r = gmr_read_counters(ws, ws_cap, &c, s)) != GMR_OK) return r;
      const int64_t tight = std::min<int64_t>((1ll << 30) - 1, (int64_t)(c.instances * 1.25) + 1024);
      if (!c.overflow && !tightened && tight < o.instance_capacity) {
        // time the candidate at the capacity it will run with (a small batch then takes the
        // one-launch list build): plan again with the measured count plus headroom
        o.instance_capacity = tight;
        tightened = true;
        continue;
      }
      if (c.overflow) {
        o.instance_capacity = std::min<int64_t>((1ll << 30) - 1, (int64_t)(c.instances * 1.25) + 1024);
        continue;
      }
      auto step = [&]() {
        gmr_status q = gmr_render_fwd(h, batch, &o, table, verts, faces, colors, rgb, nullptr, saved, ws, ws_cap, s);
        if (q == GMR_OK)
          q = gmr_render_bwd_l2(h, batch, &o, table, verts, faces, colors, rgb, target, 1.f, saved, adj_off, adj_ent,
                                recompute, dv, dc, nullptr, ws, ws_cap, s);
        return q;
      };
      if ((r = step()) != GMR_OK) return r;  // warm-up
      (void)hipEventRecord(e0, s);
      for (int i = 0; i < iters && r == GMR_OK; ++i) r = step();
      (void)hipEventRecord(e1, s);
      if (r != GMR_OK) return r;
      if (hipEventSynchronize(e1) != hipSuccess) return fail(GMR_ERR_HIP, "autotune: event sync");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_out_c = ms / (float)iters;
      o.instance_capacity = std::min<int64_t>((1ll << 30) - 1, (int64_t)(c.instances * 1.25) + 1024);
      return GMR_OK;
    }
    return GMR_ERR_CAPACITY;  // more instances than a workspace can hold: the candidate is skipped
  };
  // first pass: every candidate once; second pass: the three fastest again, each scored by the better of
  // its two timings (a candidate slowed once by interference is not lost, and a lucky first
  // timing is checked)
  struct Timed { float ms; gmr_options o; };
  std::vector<Timed> timed;
  for (const Cand& cd : cands) {
    gmr_options o = b;
    o.tile_w = cd.tw;
    o.tile_h = cd.th;
    o.px_per_lane = cd.px;
    o.raster_mode = cd.mode;
    o.lane_lists = cd.lanes;
    o.instance_capacity = std::max<int64_t>(b.instance_capacity, 1 << 20);
    float ms = 0.f;
    const gmr_status r = time_cand(o, ms);
    if (r == GMR_ERR_CAPACITY) continue;
    if ((result = r) != GMR_OK) break;
    timed.push_back({ms, o});
  }
  if (result == GMR_OK && timed.empty()) result = fail(GMR_ERR_CAPACITY, "autotune: no candidate fits 2^30 instances");
  gmr_options best = b;
  float best_ms = 1e30f;
  if (result == GMR_OK) {
    std::sort(timed.begin(), timed.end(), [](const Timed& x, const Timed& y) { return x.ms < y.ms; });
    for (size_t i = 0; i < timed.size() && i < 3 && result == GMR_OK; ++i) {
      gmr_options o = timed[i].o;
      float ms = 0.f;
      if ((result = time_cand(o, ms)) != GMR_OK) break;  // it fitted in the first pass, so it fits again
      const float score = std::min(ms, timed[i].ms);
      if (score < best_ms) {
        best_ms = score;
        best = o;
      }
    }
  }
  if (result != GMR_OK) return result;
  h->tune_cache[key] = {best, best_ms};
  *best_out = with_tuned(*base, best);
  if (ms_out) *ms_out = best_ms;
  return GMR_OK;
}

}  // extern "C"
