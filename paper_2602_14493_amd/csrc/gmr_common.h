// Internal layouts and device helpers of libgmr (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gmr.h"

namespace gmr {

constexpr int kWave = 64;            // CDNA wavefront
constexpr int kSub = 8;              // raster sub-block side: one 8x8 pixel block per wavefront
constexpr int kRecF4 = 3;            // projected record = 3 x float4 = 48 B per face-view
constexpr int kSortBlock = 512;      // onesweep workgroup (8 wavefronts)
constexpr int kScanBlock = 256;
// Onesweep elements per thread: 8 (4096-element partitions) amortises the per-partition work
// (digit descriptors, look-back) on large inputs; an input that fills fewer than 64 such
// partitions (a quarter of the CUs) takes 2 (1024), so four times as many workgroups share the
// ranking and the latency of loads and stores.  (At ~500k elements the small partitions already
// lose: their descriptors and look-back cost more than the wider spread saves.)
constexpr int kSortItemsLarge = 8, kSortItemsSmall = 2;
inline int sort_items_for(int64_t n) {
  return n < (int64_t)64 * kSortBlock * kSortItemsLarge ? kSortItemsSmall : kSortItemsLarge;
}
// Face-views per thread of the scan / emission blocks: inputs of 1M face-views or more take 8
// (2048 per block, the elements kept in registers, windowed emission); smaller ones take 4 (1024
// per block, twice the workgroups, per-lane emission).
constexpr int kScanItemsLarge = 8, kScanItemsSmall = 4;
inline int scan_items_for(int64_t n) { return n >= (int64_t{1} << 20) ? kScanItemsLarge : kScanItemsSmall; }
constexpr int kMaxPasses = 8;        // histogram rows: 0..3 depth digits (face-views), 4..7 tile digits
constexpr int kDepthPasses = 4;      // 32 depth bits in 8-bit digits
constexpr int kTileRow0 = 4;
constexpr int kHistStride = 512;     // one histogram row holds up to 512 bins
constexpr int kHistWords = kMaxPasses * kHistStride;
// The digit histograms are kept in 8 copies: workgroup b adds its counts to copy b mod 8, and a
// sort pass sums the copies of its row, so the atomics of many workgroups on few bins spread over
// 8 times as many addresses.
constexpr int kHistCopies = 8;
constexpr uint32_t kFlagAgg = 1u << 30;   // onesweep partition descriptor: aggregate published
constexpr uint32_t kFlagInc = 2u << 30;   // inclusive prefix published
constexpr uint32_t kValMask = (1u << 30) - 1u;

// Device view table --------------------------------------------------------------------------
struct TableHdr {          // 80 B
  int32_t num_views, num_meshes, tile_w, tile_h;
  int32_t tiles_total, sub_x, sub_y, items_total;   // sub_x/y: 8x8 blocks per tile; items = tiles*sub
  int64_t fv_total, pixels_total, faces_total;
  int32_t views_off, mesh_face_off, mesh_view_off, mesh_views_off;  // byte offsets in the table
  int32_t bm_shift1;  // 1 + the key bit where an instance's raster-block mask starts; 0: no masks
  int32_t pad;
};
struct ViewDev {           // 128 B
  float R[9], t[3];
  float fx, fy, cx, cy;
  int32_t W, H, tiles_x, tiles_y;
  int64_t fv_offset, pixel_offset;
  int32_t tile_base, mesh, face_begin, face_end;
  float znear, zfar;
  int32_t pad[2];
};
static_assert(sizeof(TableHdr) == 80, "table header");
static_assert(sizeof(ViewDev) == 128, "view record");

__host__ __device__ inline const ViewDev* table_views(const void* t) {
  return reinterpret_cast<const ViewDev*>(static_cast<const char*>(t) + static_cast<const TableHdr*>(t)->views_off);
}
__host__ __device__ inline const int32_t* table_i32(const void* t, int32_t off) {
  return reinterpret_cast<const int32_t*>(static_cast<const char*>(t) + off);
}

// Raster-block masks ------------------------------------------------------------------------------
// A tile of tile_w x tile_h pixels is rastered as sub_x x sub_y blocks of kSub x (tile_h / sub_y)
// pixels, block (sx, sy) being raster item sy * sub_x + sx of the tile.  When the table enables it
// (bm_shift1 > 0: the tile ids leave at least sub_x * sub_y key bits free), every sorted instance
// key carries, from bit bm_shift1 - 1 up, the mask of the tile's blocks that the instance's pixel
// rectangle meets, and a raster item reads the face-view and record of only the list entries whose
// bit it finds set (the same blocks its own rectangle test keeps).  The projection then packs,
// into each face-view element, the block column of the rectangle's left edge in its first tile
// column and of its right edge in its last, and likewise the block rows:
//   el.z = first tile | chi << 26 | rhi << 29      el.w = nx | clo << 13 | ny << 16 | rlo << 29
// (tile ids below 2^26, nx and ny below 2^13; without masks el.z is the first tile alone).
constexpr uint32_t kElTileMask = (1u << 26) - 1u;
__device__ inline uint32_t el_nx(uint32_t w) { return w & 0x1fffu; }
__device__ inline uint32_t el_ny(uint32_t w) { return (w >> 16) & 0x1fffu; }

// Blocks sx in [clo, chi], sy in [rlo, rhi] of a tile with sub_x block columns.
__device__ inline uint32_t block_mask(uint32_t clo, uint32_t chi, uint32_t rlo, uint32_t rhi, uint32_t sub_x) {
  const uint32_t cols = ((2u << chi) - 1u) & ~((1u << clo) - 1u);
  uint32_t m = 0u;
  for (uint32_t r = rlo; r <= rhi; ++r) m |= cols << (r * sub_x);
  return m;
}

// The mask of the blocks of the tile with top-left pixel (X0, Y0) that the pixel rectangle
// [ix0, ix1] x [iy0, iy1] (which meets the tile) meets.
__device__ inline uint32_t rect_block_mask(int ix0, int ix1, int iy0, int iy1, int X0, int Y0, int tw,
                                                    int tht, int sub_x, int sub_y) {
  const int bh = tht / sub_y;
  const int clo = max(ix0 - X0, 0) / kSub, chi = min(ix1 - X0, tw - 1) / kSub;
  const int rlo = max(iy0 - Y0, 0) / bh, rhi = min(iy1 - Y0, tht - 1) / bh;
  return block_mask((uint32_t)clo, (uint32_t)chi, (uint32_t)rlo, (uint32_t)rhi, (uint32_t)sub_x);
}

// Per raster item in the saved buffer (after the per-pixel state): the count and the list positions
// (16 bits each, relative to the tile's list) of the Gaussians its block composited, at most blk_cap
// = the composited_lists option of them (a larger count: the list did not fit); blk_words = 1 +
// ceil(blk_cap / 2), or 0 when none are recorded.
constexpr int kMaxCompositedLists = 8190;

// Workspace header (device counters) ------------------------------------------------------------
struct WsHdr {                 // 256 B at the start of the workspace
  uint32_t count;              // instances generated (may exceed capacity)
  uint32_t overflow;
  uint32_t capacity;
  uint32_t passes;
  uint32_t part_ctr[kMaxPasses];   // onesweep partition tickets, one per pass (same rows as the histograms)
  uint32_t stats_items;            // raster items; each writes its own statistics slot
  uint32_t bwd_stats;              // 1 once a backward has written its per-item slots
  unsigned long long stats_fwd_off;  // byte offset in the workspace: [items] u64 pairs of the forward
  unsigned long long stats_bwd_off;  // [items] float4 {colour loss, silhouette loss, pairs lo, hi} of the backward
  float loss;                      // colour loss of the last fused backward (fixed-order sum of the slots)
  float loss_sil;                  // its silhouette loss
  uint32_t red_ticket;             // last-block ticket of that sum (left at 0)
  // range of the high 16 depth-key bits over visible face-views, in kKeyCopies copies (projection
  // workgroup b folds its range into copy b mod kKeyCopies; readers combine the copies)
  uint32_t key_hi_min[8], key_hi_max[8];
  uint32_t emit_ctr;               // block tickets of the one-pass scan + emission
  uint32_t peak_count;             // largest instance count of any list build since it was last reset
                                   // (by gmr_read_counters; zeroed with the header by the caller)
  uint32_t pad1[25];
};
static_assert(sizeof(WsHdr) == 256, "ws header");

// Silhouette term: alpha is clamped to [kBceEps, 1 - kBceEps] inside the binary cross-entropy.
constexpr float kBceEps = 1e-6f;

// When the visible face-views' depth keys span fewer than 256 values of their high 16 bits, the
// third depth pass sorts on (key >> 16) - key_hi_min (one 8-bit digit that orders them exactly)
// and the fourth pass is skipped; the sorted elements then end in the second element buffer.
// Culled face-views (key 0xffffffff, no instances) may land anywhere: they emit nothing.
constexpr int kKeyCopies = 8;
__device__ inline uint32_t key_hi_min(const WsHdr* h) {
  uint32_t m = h->key_hi_min[0];
#pragma unroll
  for (int c = 1; c < kKeyCopies; ++c) m = min(m, h->key_hi_min[c]);
  return m;
}
__device__ inline bool depth_keys_narrow(const WsHdr* h) {
  uint32_t mx = h->key_hi_max[0];
#pragma unroll
  for (int c = 1; c < kKeyCopies; ++c) mx = max(mx, h->key_hi_max[c]);
  const uint32_t mn = key_hi_min(h);
  return mx >= mn && mx - mn < 256u;
}

// Kernel-side options (plain values) ---------------------------------------------------------------
struct KOpts {
  int32_t cov_mode;
  float dilation, alpha_min, alpha_max, t_eps;
  float bg0, bg1, bg2;
  int32_t sh_degree;  // view-dependent colour degree (0: Eq. 16)
  uint32_t blk_words; // words per raster item of the composited lists (0: none)
  uint32_t blk_cap;   // list positions per raster item
};

// Where the per-item raster statistics live (recorded in the header by the build prologue).
struct StatsInfo {
  uint32_t items;
  unsigned long long fwd_off, bwd_off;
  uint32_t bwd;  // 1: a backward follows in the same call (its counters are set up with the lists)
};

// Blocks of the fixed-order loss sum (a multiple of nothing in particular; at most this many).
constexpr int kLossReduceBlocks = 256;

// Workspace layout, computed on the host (byte offsets) -------------------------------------------
struct Layout {
  size_t hdr, rec, elA, elB, bdesc, instA, instB, keysF, valsF, hist, descF0, descF1, descI0, descI1,
      ranges, dfv, fgrad, fsh, statF, statB, statR, total;
  int64_t fv_total, faces_total, pixels_total, capacity;
  int32_t tiles_total, items_total, tile_bits, tile_passes, scan_blocks, parts_fv, parts_inst;
  int32_t scan_items;  // face-views per thread of the scan / emission blocks (scan_items_for)
  int32_t sort_items_fv, sort_items_inst;  // onesweep elements per thread (sort_items_for)
  int32_t tile_shift[kMaxPasses - kTileRow0], tile_mask[kMaxPasses - kTileRow0];
};

// Small device helpers -------------------------------------------------------------------------------
__device__ inline float u2f(uint32_t x) { return __uint_as_float(x); }
__device__ inline uint32_t f2u(float x) { return __float_as_uint(x); }

__device__ inline uint64_t ballot64(bool p) { return __ballot(p); }

__device__ inline void wave_lds_sync() {
  // LDS requests of one wavefront complete in order; this keeps the compiler from reordering an
  // LDS store of one lane past a later LDS load of another lane.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Mesh containing global face f (face offsets are ascending).
__device__ inline int find_mesh(const int32_t* mesh_face_off, int num_meshes, int32_t f) {
  int lo = 0, hi = num_meshes - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (mesh_face_off[mid] <= f) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Digit layout of the instance (tile-id) passes: pass p sorts (tile >> shift[p]) & mask[p].
struct TilePasses {
  int n;
  int shift[kMaxPasses - kTileRow0];
  uint32_t mask[kMaxPasses - kTileRow0];
};

// View containing face-view fv (face-view offsets are ascending).
__device__ inline int find_view_by_fv(const ViewDev* views, int nv, int64_t fv) {
  int lo = 0, hi = nv - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].fv_offset <= fv) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// View containing global tile t (tile bases are ascending).
__device__ inline int find_view_by_tile(const ViewDev* views, int nv, int32_t t) {
  int lo = 0, hi = nv - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_base <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Conversion of one face (Sec. 2.2) in closed form, double precision.  The uniform triangle's
// covariance sum_q (q - mu)(q - mu)^T / 12 written with the edges e1 = v_j - v_i, e2 = v_k - v_i
// is C = (2 e1 e1^T + 2 e2 e2^T - e1 e2^T - e2 e1^T) / 36: the embedded 2D covariance of Eq. 15.
// Eq. 13 scales it by kappa = |A| / (pi sqrt(max(lambda1 lambda2, eps))) with lambda1 lambda2 =
// |A|^2 / 108 and adds s_z^2 n n^T.
// cov_mode 2 is the "3DGS-based" baseline of Sec. 3.1 (Baselines): rotation from the normal (z)
// and the first edge (x = e1 / |e1|, y = n x x), scales read as kappa C's variances along x and y
// and s_z along n: S = kappa (x'Cx) x x' + kappa (y'Cy) y y' + s_z^2 n n'.
struct FaceGeo {
  double e1[3], e2[3], m[3];   // edges and their cross product
  double mm, area, kappa;      // |m|, |A|, kappa (1 in the embedded form)
  bool clamped;                // kappa from the epsilon branch of Eq. 12
  double mu[3];
  double S[6];                 // xx xy xz yy yz zz
};

constexpr double kPi = 3.14159265358979323846;
constexpr double kEpsL = 1e-14;   // Eq. 12
constexpr double kSz2 = 1e-12;    // s_z^2, s_z = 1e-6

__device__ inline bool face_convert(const double* vi, const double* vj, const double* vk, int cov_mode, FaceGeo& g) {
  for (int a = 0; a < 3; ++a) { g.e1[a] = vj[a] - vi[a]; g.e2[a] = vk[a] - vi[a]; }
  g.m[0] = g.e1[1] * g.e2[2] - g.e1[2] * g.e2[1];
  g.m[1] = g.e1[2] * g.e2[0] - g.e1[0] * g.e2[2];
  g.m[2] = g.e1[0] * g.e2[1] - g.e1[1] * g.e2[0];
  double mm2 = g.m[0] * g.m[0] + g.m[1] * g.m[1] + g.m[2] * g.m[2];
  if (!(mm2 > 0.0) || !(mm2 < 1e300)) return false;
  g.mm = sqrt(mm2);
  g.area = 0.5 * g.mm;
  for (int a = 0; a < 3; ++a) g.mu[a] = (vi[a] + vj[a] + vk[a]) * (1.0 / 3.0);
  const double* e1 = g.e1;
  const double* e2 = g.e2;
  double M[6];
  M[0] = 2.0 * e1[0] * e1[0] + 2.0 * e2[0] * e2[0] - 2.0 * e1[0] * e2[0];
  M[1] = 2.0 * e1[0] * e1[1] + 2.0 * e2[0] * e2[1] - e1[0] * e2[1] - e2[0] * e1[1];
  M[2] = 2.0 * e1[0] * e1[2] + 2.0 * e2[0] * e2[2] - e1[0] * e2[2] - e2[0] * e1[2];
  M[3] = 2.0 * e1[1] * e1[1] + 2.0 * e2[1] * e2[1] - 2.0 * e1[1] * e2[1];
  M[4] = 2.0 * e1[1] * e1[2] + 2.0 * e2[1] * e2[2] - e1[1] * e2[2] - e2[1] * e1[2];
  M[5] = 2.0 * e1[2] * e1[2] + 2.0 * e2[2] * e2[2] - 2.0 * e1[2] * e2[2];
  if (cov_mode == 1) {
    g.kappa = 1.0;
    g.clamped = false;
    for (int a = 0; a < 6; ++a) g.S[a] = M[a] * (1.0 / 36.0);
    return true;
  }
  double det2 = g.area * g.area * (1.0 / 108.0);
  g.clamped = !(det2 >= kEpsL);
  g.kappa = g.area / (kPi * sqrt(g.clamped ? kEpsL : det2));
  double inv = 1.0 / g.mm;
  double n0 = g.m[0] * inv, n1 = g.m[1] * inv, n2 = g.m[2] * inv;
  if (cov_mode == 2) {
    const double il = 1.0 / sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    const double x[3] = {e1[0] * il, e1[1] * il, e1[2] * il};
    const double y[3] = {n1 * x[2] - n2 * x[1], n2 * x[0] - n0 * x[2], n0 * x[1] - n1 * x[0]};
    const double xMx = M[0] * x[0] * x[0] + M[3] * x[1] * x[1] + M[5] * x[2] * x[2] +
                       2.0 * (M[1] * x[0] * x[1] + M[2] * x[0] * x[2] + M[4] * x[1] * x[2]);
    const double yMy = M[0] * y[0] * y[0] + M[3] * y[1] * y[1] + M[5] * y[2] * y[2] +
                       2.0 * (M[1] * y[0] * y[1] + M[2] * y[0] * y[2] + M[4] * y[1] * y[2]);
    const double sx2 = g.kappa * xMx * (1.0 / 36.0), sy2 = g.kappa * yMy * (1.0 / 36.0);
    const double n[3] = {n0, n1, n2};
    const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
    for (int a = 0; a < 6; ++a)
      g.S[a] = sx2 * x[rr[a]] * x[cc[a]] + sy2 * y[rr[a]] * y[cc[a]] + kSz2 * n[rr[a]] * n[cc[a]];
    return true;
  }
  double k36 = g.kappa * (1.0 / 36.0);
  g.S[0] = k36 * M[0] + kSz2 * n0 * n0;
  g.S[1] = k36 * M[1] + kSz2 * n0 * n1;
  g.S[2] = k36 * M[2] + kSz2 * n0 * n2;
  g.S[3] = k36 * M[3] + kSz2 * n1 * n1;
  g.S[4] = k36 * M[4] + kSz2 * n1 * n2;
  g.S[5] = k36 * M[5] + kSz2 * n2 * n2;
  return true;
}

// EWA projection of (mu, S) through view V, double precision (Sec. 2.1's splatting: first-order
// Jacobian of the pinhole at the mean; a `dilation` px^2 low-pass on the screen covariance).
struct ProjGeo {
  double p[3];         // camera-space mean
  double J[6];         // 2x3 Jacobian of (u, v) w.r.t. p
  double W[6];         // R S R^T (xx xy xz yy yz zz)
  double sxx, sxy, syy, det;
  double a, b, c;      // conic = inverse screen covariance
  double u, v;
};

__device__ inline bool view_project(const ViewDev& V, const double* mu, const double* S, double dilation, ProjGeo& q) {
  for (int r = 0; r < 3; ++r)
    q.p[r] = (double)V.R[3 * r] * mu[0] + (double)V.R[3 * r + 1] * mu[1] + (double)V.R[3 * r + 2] * mu[2] + (double)V.t[r];
  if (!(q.p[2] > (double)V.znear) || !(q.p[2] < (double)V.zfar)) return false;
  double iz = 1.0 / q.p[2];
  double fx = V.fx, fy = V.fy;
  q.J[0] = fx * iz; q.J[1] = 0.0; q.J[2] = -fx * q.p[0] * iz * iz;
  q.J[3] = 0.0; q.J[4] = fy * iz; q.J[5] = -fy * q.p[1] * iz * iz;
  // W = R S R^T with S symmetric (xx xy xz yy yz zz)
  double Sf[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
  double RS[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      RS[3 * r + c] = (double)V.R[3 * r] * Sf[c] + (double)V.R[3 * r + 1] * Sf[3 + c] + (double)V.R[3 * r + 2] * Sf[6 + c];
  double Wf[9];
  for (int r = 0; r < 3; ++r)
    for (int c = r; c < 3; ++c)
      Wf[3 * r + c] = RS[3 * r] * (double)V.R[3 * c] + RS[3 * r + 1] * (double)V.R[3 * c + 1] + RS[3 * r + 2] * (double)V.R[3 * c + 2];
  q.W[0] = Wf[0]; q.W[1] = Wf[1]; q.W[2] = Wf[2]; q.W[3] = Wf[4]; q.W[4] = Wf[5]; q.W[5] = Wf[8];
  // J W J^T with J = [[j0 0 j2],[0 j4 j5]]
  double w00 = q.W[0], w01 = q.W[1], w02 = q.W[2], w11 = q.W[3], w12 = q.W[4], w22 = q.W[5];
  double j0 = q.J[0], j2 = q.J[2], j4 = q.J[4], j5 = q.J[5];
  double t0 = j0 * w00 + j2 * w02, t1 = j0 * w01 + j2 * w12, t2 = j0 * w02 + j2 * w22;   // row 0 of J W
  double s1 = j4 * w11 + j5 * w12, s2 = j4 * w12 + j5 * w22;                               // row 1 (cols 1,2)
  q.sxx = t0 * j0 + t2 * j2 + dilation;
  q.sxy = t1 * j4 + t2 * j5;
  q.syy = s1 * j4 + s2 * j5 + dilation;
  q.det = q.sxx * q.syy - q.sxy * q.sxy;
  if (!(q.det > 0.0)) return false;
  double id = 1.0 / q.det;
  q.a = q.syy * id;
  q.b = -q.sxy * id;
  q.c = q.sxx * id;
  q.u = fx * q.p[0] * iz + (double)V.cx;
  q.v = fy * q.p[1] * iz + (double)V.cy;
  return true;
}

// exp(power) = exp2(-(k w)^2) with w = L (dx, dy), L^T L = conic, k^2 = log2(e) / 2.
constexpr double kHalfLog2e = 0.72134752044448170368;    // log2(e) / 2
constexpr double kRasterScale = 0.84932180028801904272;  // k = sqrt(log2(e) / 2), the records' scale of L
constexpr double kLn2 = 0.69314718055994530942;

// Pixel-centre predicate of the 3-sigma extent, per axis: the pixels i with |i + 0.5 - u| <= r
// are ceil(u - r - 0.5) .. floor(u + r - 0.5) (computed in double by the projection).

}  // namespace gmr
