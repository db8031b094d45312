// Per-tile front-to-back alpha compositing and its reverse-order adjoint (the 3DGS rasteriser of
// Sec. 2.1, with opacity 1 per Sec. 2.2's colour assignment).
//
// Work item = one 8 x (8 PX) pixel block of a tile, handled by one wavefront: lane (lx, ly) owns the
// PX pixels (lx, ly + 8k), k < PX.  A wavefront walks its tile's depth-sorted list 64 instances at
// a time: each lane gathers one 48 B record, the records whose integer pixel rectangle meets the
// block are kept (ballot), staged in the wavefront's LDS slots and consumed in list order as
// wave-uniform broadcasts; the x offset and x extent test of a lane are shared by its PX pixels.
// The wavefront leaves as soon as every pixel has stopped.  Wavefronts never synchronise with each
// other, so a tile's blocks finish independently.  With per-lane lists (forward only), the staged
// batch's pixel-rectangle coverage of the block is transposed across the wavefront so that each
// lane walks only the Gaussians over its own pixel: same pairs, same arithmetic, fewer idle lanes.
//
// Per pixel and Gaussian (exp(power) = exp2(-(w1^2 + w2^2)), w = k L (dx, dy), L^T L = conic):
//   inside = pixel in the Gaussian's 3-sigma pixel rectangle
//   alpha  = min(alpha_max, exp(power)); skipped when alpha < alpha_min
//   stop (without compositing) when T (1 - alpha) < t_eps; else C += c alpha T, T *= 1 - alpha
// Saved per pixel: T_final and the list position after the last composited Gaussian.
//
// Backward, per pixel from that position down to the list start:
//   T_k = T_{k+1} / (1 - alpha_k)
//   dL/dalpha_k = T_k (c_k . g_C) - (S_k + T_f (bg . g_C) - T_f g_A) / (1 - alpha_k),
//   S_k = sum over later composited j of alpha_j T_j (c_j . g_C)
//   dL/dpower = alpha dL/dalpha when unclamped, else 0
//   (du, dv) = -dL/dpower (conic (dx, dy));  (da, db, dc) = -dL/dpower (dx^2/2, dx dy, dy^2/2)
//   dL/dc_k = alpha_k T_k g_C
// A lane first sums its PX pixels' partials; the 8 sums are then reduced over the wavefront by a
// transposed butterfly that halves the values carried per lane at each of the first three steps
// (half-wave and row swaps, then DPP), and 8 lanes issue one float atomic each into the
// face-view's gradient record.  Gaussians that no pixel of a row group reaches, or that no pixel
// composites, are skipped wave-uniformly.
#include "gmr_common.h"
#include "gmr_launch.h"

namespace gmr {

// blockIdx -> work group such that each of the 8 XCDs (blocks are dealt round-robin to them)
// receives a contiguous run of tiles: neighbouring tiles share Gaussians, which then share an L2.
__device__ inline int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

struct ItemGeo {
  int tile, sub, x, bx0, by0, W, H;  // sub: the block's index among its tile's raster items
  bool any;
  int64_t row0;  // pixel index of (0, by0 + ly) in the flat image
};

template <int PX>
__device__ inline ItemGeo item_geometry(const TableHdr* th, const ViewDev* views, int item, int lane) {
  item = __builtin_amdgcn_readfirstlane(item);  // one item per wavefront: keep its geometry scalar
  ItemGeo g;
  const int spt = th->sub_x * th->sub_y;
  g.tile = item / spt;
  const int sub = item - g.tile * spt;
  g.sub = sub;
  const int vi = find_view_by_tile(views, th->num_views, g.tile);
  const ViewDev& V = views[vi];
  const int lt = g.tile - V.tile_base;
  const int tyi = lt / V.tiles_x, txi = lt - tyi * V.tiles_x;
  const int sy = sub / th->sub_x, sx = sub - sy * th->sub_x;
  g.bx0 = txi * th->tile_w + sx * kSub;
  g.by0 = tyi * th->tile_h + sy * (kSub * PX);
  g.W = V.W;
  g.H = V.H;
  g.any = g.bx0 < V.W && g.by0 < V.H;
  g.x = g.bx0 + (lane & 7);
  g.row0 = V.pixel_offset + (int64_t)(g.by0 + (lane >> 3)) * V.W;
  return g;
}

// Key bit of this item's block in the instances' raster-block masks, or -1 without masks (then every
// list entry is tested against the block's rectangle).
__device__ inline int item_key_bit(const TableHdr* th, const ItemGeo& g) {
  return th->bm_shift1 > 0 ? th->bm_shift1 - 1 + g.sub : -1;
}

__device__ inline bool rect_meets_block(uint32_t rx, uint32_t ry, int bx0, int by0, int bh) {
  const int ix0 = (int)(rx & 0xffffu), ix1 = (int)(rx >> 16), iy0 = (int)(ry & 0xffffu), iy1 = (int)(ry >> 16);
  return ix0 <= bx0 + kSub - 1 && ix1 >= bx0 && iy0 <= by0 + bh - 1 && iy1 >= by0;
}

// Whether the record's Gaussian can reach the alpha cutoff anywhere in the pixel-centre box of the
// block [bx0 + 1/2, bx0 + 7.5] x [by0 + 1/2, by0 + bh - 1/2]: the minimum over that box of its
// power (w1^2 + w2^2 of gauss_exp, a convex quadratic in the offset) against pmax.  The minimum is 0
// when the mean is inside the box, else it lies on an edge, where the quadratic is minimised in
// closed form and clamped to the edge.  The box holds every pixel centre of the block, so a record
// rejected here composites at none of them (pmax carries a margin over the cutoff's power).
__device__ inline bool ellipse_meets_block(const float4& r0, const float4& r1, int bx0, int by0, int bh, float pmax) {
  const float cx = r0.x + r0.z, cy = r0.y + r0.w;
  const float lox = ((float)bx0 + 0.5f) - cx, hix = ((float)bx0 + (float)(kSub - 1) + 0.5f) - cx;
  const float loy = ((float)by0 + 0.5f) - cy, hiy = ((float)(by0 + bh - 1) + 0.5f) - cy;
  if (lox <= 0.f && hix >= 0.f && loy <= 0.f && hiy >= 0.f) return true;
  const float l11 = r1.x, l12 = r1.y, l22 = r1.z;
  const float cyy = fmaf(l12, l12, l22 * l22);  // coefficient of dy^2
  auto power = [&](float dx, float dy) {
    const float w1 = fmaf(l11, dx, l12 * dy), w2 = l22 * dy;
    return fmaf(w1, w1, w2 * w2);
  };
  // edges dx = const: minimiser dy = -l11 l12 dx / cyy; edges dy = const: dx = -l12 dy / l11
  const float ky = -(l11 * l12) / cyy, kx = -l12 / l11;
  const float p1 = power(lox, fminf(fmaxf(ky * lox, loy), hiy));
  const float p2 = power(hix, fminf(fmaxf(ky * hix, loy), hiy));
  const float p3 = power(fminf(fmaxf(kx * loy, lox), hix), loy);
  const float p4 = power(fminf(fmaxf(kx * hiy, lox), hix), hiy);
  return fminf(fminf(p1, p2), fminf(p3, p4)) <= pmax;
}

// Pixels of an 8 x 8 block (bit 8 * row + col) at whose centre the Gaussian's power is at most pmax:
// pixel (c, r) takes dx = ox - c, dy = oy - r (offsets as staged), and the power is at most pmax
// exactly where |l11 dx + l12 dy| <= sqrt(pmax - (l22 dy)^2), i.e. for c within
// ox + (l12 dy -/+ sqrt(pmax - (l22 dy)^2)) / l11.  Records are finite with l11 > 0 (the projection
// writes none other).  The half-width is widened by 1e-3 px, which covers the hardware square
// root's and reciprocal's rounding; with pmax carrying a margin over the power of the alpha cutoff,
// every pixel at which the record reaches alpha_min is inside, so masking a walk with it changes no
// image.  Each bound is clamped to the block before it is converted; an empty range gives no bits.
__device__ inline uint64_t ellipse_rows(float ox, float oy, float l11, float l12, float l22, float pmax) {
  const float il = __builtin_amdgcn_rcpf(l11);
  const float w2o = l22 * oy, l12o = l12 * oy;
  uint32_t m[2] = {0u, 0u};
#pragma unroll
  for (int r = 0; r < kSub; ++r) {
    const float w2 = fmaf(-l22, (float)r, w2o);  // l22 dy
    const float t = fmaf(-w2, w2, pmax);
    const float hw = fmaf(__builtin_amdgcn_sqrtf(fmaxf(t, 0.f)), il, 1e-3f);
    const float c = fmaf(fmaf(-l12, (float)r, l12o), il, ox);
    const int ilo = (int)ceilf(__builtin_amdgcn_fmed3f(c - hw, 0.f, 8.f));    // 0 .. 8
    const int ihi = (int)floorf(__builtin_amdgcn_fmed3f(c + hw, -1.f, 7.f));  // -1 .. 7
    const uint32_t bits = (0xFFu << ilo) & (0xFFu >> (kSub - 1 - ihi));        // 0 when ilo > ihi
    m[r >> 2] |= (t >= 0.f ? bits : 0u) << (kSub * (r & 3));
  }
  return (uint64_t)m[0] | ((uint64_t)m[1] << 32);
}

__device__ inline bool in_range(uint32_t r, int x) {
  const int lo = (int)(r & 0xffffu), hi = (int)(r >> 16);
  return (uint32_t)(x - lo) <= (uint32_t)(hi - lo);
}

// Shared by forward and backward so both take bit-identical decisions: w = k L (dx, dy) with the
// record's scaled Cholesky factor (l11, l12, l22), exp(power) = exp2(-(w1^2 + w2^2)).
__device__ inline float gauss_exp(float l11, float l12, float l22, float dx, float dy, float& w1, float& w2) {
  w1 = fmaf(l11, dx, l12 * dy);
  w2 = l22 * dy;
  return __builtin_amdgcn_exp2f(-fmaf(w1, w1, w2 * w2));
}

// A record as a wavefront stages it for its block: the mean as offsets from the centre of an
// 8 x 8 block's top-left pixel (origin bx0 or yb), with the mean's low half folded in, so that
// pixel (bx0 + c, yb + r) of that block takes dx = ox - c and dy = oy - r.  Forward and backward
// stage and subtract the same way, so they take the same decisions; the offsets depend on the
// 8 x 8 block alone (never on the tile shape or the pixels per lane), so neither do images.
// LDS slot j: s[0] = {ox, oy of row group 0, l11, l12}, s[1] = {l22, r, g, b} and, with PX > 1
// row groups, s[2] = {oy of row groups 1, 2, 3, 0}.
__device__ inline float block_off(float hi, float lo, int origin) { return (hi - ((float)origin + 0.5f)) + lo; }

template <int PX>
__device__ inline void stage_record(float4 (*s)[kWave], int slot, const float4& r0, const float4& r1,
                                    const float4& r2, int bx0, int by0) {
  s[0][slot] = make_float4(block_off(r0.x, r0.z, bx0), block_off(r0.y, r0.w, by0), r1.x, r1.y);
  s[1][slot] = make_float4(r1.z, r2.x, r2.y, r2.z);
  if constexpr (PX > 1)
    s[2][slot] = make_float4(block_off(r0.y, r0.w, by0 + kSub), PX > 2 ? block_off(r0.y, r0.w, by0 + 2 * kSub) : 0.f,
                             PX > 2 ? block_off(r0.y, r0.w, by0 + 3 * kSub) : 0.f, 0.f);
}

// The row-group offsets oy of staged slot j (a = s[0][j]).
template <int PX>
__device__ __forceinline__ void staged_oy(const float4 (*s)[kWave], int j, const float4& a, float (&oy)[PX]) {
  oy[0] = a.y;
  if constexpr (PX > 1) {
    const float4 c = s[2][j];
    oy[1] = c.x;
    if constexpr (PX > 2) {
      oy[2] = c.y;
      oy[3] = c.z;
    }
  }
}

// DPP controls (GFX9 encoding): quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror, row_ror:8,
// row_shl:4 (lane i reads i + 4 of its 16-lane row), row_shr:4 (reads i - 4).
constexpr int kDppXor1 = 0xB1;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppRowRor8 = 0x128;
constexpr int kDppRowShl4 = 0x104;
constexpr int kDppRowShr4 = 0x114;

// v + (v read from the lane that DPP control kCtrl selects inside its 16-lane row); the
// permute folds into the add as a DPP operand modifier
template <int kCtrl>
__device__ __forceinline__ float add_dpp(float acc, float v) {
  return acc + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, true));
}

// The value lane ^ B holds, B in {1, 2, 4, 8, 16}.  All lanes must be active.  up: all ones in the
// lanes with (lane & B) set, else 0.
template <int B>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, uint32_t up) {
  if constexpr (B == 1) return __builtin_amdgcn_update_dpp(0u, v, kDppXor1, 0xF, 0xF, true);
  else if constexpr (B == 2) return __builtin_amdgcn_update_dpp(0u, v, kDppXor2, 0xF, 0xF, true);
  else if constexpr (B == 4) {
    // banks 0 and 2 of each row (lane bit 2 clear) read lane + 4, banks 1 and 3 read lane - 4
    const uint32_t t = __builtin_amdgcn_update_dpp(0u, v, kDppRowShl4, 0xF, 0x5, true);
    return __builtin_amdgcn_update_dpp(t, v, kDppRowShr4, 0xF, 0xA, false);
  } else if constexpr (B == 8) return __builtin_amdgcn_update_dpp(0u, v, kDppRowRor8, 0xF, 0xF, true);
  else {
    static_assert(B == 16, "lane_xor: B in {1, 2, 4, 8, 16}");
    // swapping the odd rows of one copy with the even rows of another leaves row r's partner row
    // in the first copy for odd r and in the second for even r
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (r[0] & up) | (r[1] & ~up);
  }
}

// One step of the 64 x 64 bit transpose on one 32-bit word: rows (lanes) r and r ^ B exchange the
// off-diagonal B x B blocks; m selects the bit positions p with (p & B) == 0.  A lane without B
// keeps its m bits and takes the partner's m bits shifted up by B; a lane with B keeps its ~m bits
// and takes the partner's ~m bits shifted down -- written with masks, not branches (every lane
// runs the same instructions, as the lane exchanges need).
template <int B>
__device__ __forceinline__ uint32_t transpose_step(uint32_t w, uint32_t m) {
  const uint32_t up = 0u - ((__lane_id() >> __builtin_ctz(B)) & 1u);
  const uint32_t y = lane_xor<B>(w, up);
  const uint32_t sh = ((y >> B) & up) | ((y << B) & ~up);
  const uint32_t keep = m ^ up;
  return (w & keep) | (sh & ~keep);
}

// Lane r holds row r of a 64 x 64 bit matrix (bit c = entry (r, c)); returns column `lane`.
__device__ inline uint64_t transpose64(uint64_t x, int lane) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  // B = 32: lanes 0-31 keep their low words and take the partner's low word as the high word;
  // lanes 32-63 keep their high words and take the partner's high word as the low word -- one
  // half-wave swap of the low words of the upper half with the high words of the lower half
  const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
  lo = r[0];
  hi = r[1];
  lo = transpose_step<16>(lo, 0x0000FFFFu); hi = transpose_step<16>(hi, 0x0000FFFFu);
  lo = transpose_step<8>(lo, 0x00FF00FFu);  hi = transpose_step<8>(hi, 0x00FF00FFu);
  lo = transpose_step<4>(lo, 0x0F0F0F0Fu);  hi = transpose_step<4>(hi, 0x0F0F0F0Fu);
  lo = transpose_step<2>(lo, 0x33333333u);  hi = transpose_step<2>(hi, 0x33333333u);
  lo = transpose_step<1>(lo, 0x55555555u);  hi = transpose_step<1>(hi, 0x55555555u);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Pixels of the 8 x 8 block at (bx0, yb) inside the integer rectangle (rx, ry): bit 8 * row + col.
__device__ inline uint64_t block_coverage(uint32_t rx, uint32_t ry, int bx0, int yb) {
  const int c0 = max((int)(rx & 0xffffu) - bx0, 0), c1 = min((int)(rx >> 16) - bx0, kSub - 1);
  const int r0 = max((int)(ry & 0xffffu) - yb, 0), r1 = min((int)(ry >> 16) - yb, kSub - 1);
  if (c0 > c1 || r0 > r1) return 0ull;
  const uint32_t cols = (0xFFu << c0) & (0xFFu >> (kSub - 1 - c1));
  const uint32_t rep = cols * 0x01010101u;
  const uint64_t rows = (~0ull << (8 * r0)) & (~0ull >> (8 * (kSub - 1 - r1)));
  return (((uint64_t)rep << 32) | rep) & rows;
}

__device__ __forceinline__ int ctz64(uint64_t m) { return __builtin_ctzll(m); }

// ------------------------------------------------------------------------------------------------
// forward
// ------------------------------------------------------------------------------------------------
struct FwdArgs {
  const void* table;
  const uint32_t* ranges;
  const uint32_t* vals;
  const uint32_t* keys;  // sorted keys: tile id and, above it, the raster-block mask
  const float4* rec;
  KOpts o;
  float* out_rgb;
  float* out_alpha;
  float* saved_T;
  uint32_t* saved_n;
  uint32_t* blk;              // [items][o.blk_words] composited lists (see blk_append), or NULL
  unsigned long long* stats;  // [items] pairs evaluated per item (summed on the host when read)
};

// One list entry as a lane holds it: its key and face-view.  The raster loops load the next batch of
// 64 entries while they work on the current one; positions are relative to the list's start (keys
// and vals point there), and one outside the non-empty window [0, len) reads its nearest entry
// instead, so that the loads need no branch (the caller ignores it) and the compiler can wait for
// exactly the batch it uses.
struct Entry {
  uint32_t key, id;
};
__device__ __forceinline__ Entry load_entry(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                            int32_t r, int32_t len) {
  const int32_t q = min(max(r, 0), len - 1);
  return Entry{keys[q], vals[q]};
}

// Whether an entry may meet the item's block: with masks its key bit, else the rectangle test on
// the record's two rectangle words.
template <int PX>
__device__ __forceinline__ bool entry_kept(const Entry& e, int kbit, const float4* __restrict__ rec,
                                           const ItemGeo& g) {
  if (kbit >= 0) return ((e.key >> kbit) & 1u) != 0u;
  const float4* rp = rec + (size_t)kRecF4 * e.id;
  return rect_meets_block(f2u(rp[1].w), f2u(rp[2].w), g.bx0, g.by0, kSub * PX);
}

// The item's composited list in the saved buffer, or NULL when none is recorded: no buffer, or a tile
// list longer than 16-bit positions reach (its count is then set to 0xffffffff, "did not fit").
__device__ __forceinline__ uint32_t* blk_of(const FwdArgs& a, int item, uint32_t len, int lane) {
  if (!a.blk) return nullptr;
  uint32_t* const g = a.blk + (size_t)item * a.o.blk_words;
  if (len <= 65536u) return g;
  if (lane == 0) g[0] = ~0u;
  return nullptr;
}

// A block's composited list.  Per raster item the forward records, in list order, the list positions
// (relative to the tile's list start) of the Gaussians that at least one of its pixels composited:
// word 0 the count, then the positions as 16-bit values, o.blk_cap of them at most (those past the
// count undefined; a count above the cap means the list did not fit, and a tile list longer than
// 65536 entries records no list: count 0xffffffff).  The backward walks only these -- a Gaussian
// no pixel of the block composited adds nothing to the block's gradients -- instead of testing
// every entry of the tile's list against the block.  Appends the staged slots set in the wave-uniform mask M (slot j
// at list position pos_j), in slot order, to the item's list g.
__device__ __forceinline__ void blk_append(uint32_t* g, uint32_t cap, uint64_t M, uint32_t pos_lane, uint32_t& cnt,
                                           int lane) {
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if ((M >> lane) & 1ull) {
    const uint32_t idx = cnt + (uint32_t)__popcll(M & below);
    if (idx < cap) reinterpret_cast<uint16_t*>(g + 1)[idx] = (uint16_t)pos_lane;
  }
  cnt += (uint32_t)__popcll(M);
}

// One record against a lane's PX pixels; `valid` = false makes it a no-op (predicated).  a = s[0][j],
// b = s[1][j]; cov[k]: the record's pixel-rectangle coverage of row group k (bit = lane), uniform.
template <int PX>
__device__ __forceinline__ bool fwd_eval(const float4& a, const float4& b, const float (&oy)[PX],
                                         const uint64_t (&cov)[PX], bool valid, uint32_t pos_next, float lxf,
                                         float lyf, float amin, float amax, float teps, float (&T)[PX],
                                         float (&C0)[PX], float (&C1)[PX], float (&C2)[PX], uint32_t (&last)[PX],
                                         bool (&done)[PX], unsigned long long& pairs) {
  const float dx = a.x - lxf;
  bool any = false;  // some pixel composited it
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const bool act = valid && !done[k] && __builtin_amdgcn_inverse_ballot_w64(cov[k]);
    if (PX > 1 && __ballot(act) == 0ull) continue;  // wave-uniform: no lane's row k meets it
    const float dy = oy[k] - lyf;
    float w1, w2;
    const float e = gauss_exp(a.z, a.w, b.x, dx, dy, w1, w2);
    const float al = __builtin_amdgcn_fmed3f(e, 0.f, amax);  // min(e, amax): e is in [0, 1]
    const bool ok = act && al >= amin;
    const float Tn = T[k] * (1.f - al);
    const bool stop = ok && Tn < teps;
    const bool comp = ok && !(Tn < teps);
    any = any || comp;
    pairs += (unsigned long long)__popcll(__ballot(act));  // wave-uniform, scalar unit
    done[k] = done[k] || stop;
    const float wt = al * T[k];
    C0[k] = comp ? fmaf(b.y, wt, C0[k]) : C0[k];
    C1[k] = comp ? fmaf(b.z, wt, C1[k]) : C1[k];
    C2[k] = comp ? fmaf(b.w, wt, C2[k]) : C2[k];
    T[k] = comp ? Tn : T[k];
    last[k] = comp ? pos_next : last[k];
  }
  return __ballot(any) != 0ull;  // wave-uniform
}

// A wave-uniform 64-bit value from LDS into scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Returns the item's pair count (wave-uniform).
template <int PX>
__device__ inline unsigned long long raster_fwd_item(const FwdArgs& a, const TableHdr* th, const ViewDev* views,
                                                     int item, int lane, float4 (*s)[kWave], uint64_t (*scov)[kWave],
                                                     uint32_t& bcnt) {
  item = __builtin_amdgcn_readfirstlane(item);
  const ItemGeo g = item_geometry<PX>(th, views, item, lane);
  if (!g.any) {  // a block past the image's edge composites nothing
    if (a.blk && lane == 0) a.blk[(size_t)item * a.o.blk_words] = 0u;
    return 0ull;
  }
  const int ly = lane >> 3;
  const float lxf = (float)(lane & 7), lyf = (float)ly;
  const uint32_t start = a.ranges[2 * (size_t)g.tile], end = a.ranges[2 * (size_t)g.tile + 1];
  const float amin = a.o.alpha_min, amax = a.o.alpha_max, teps = a.o.t_eps;
  const float pmax = -__builtin_amdgcn_logf(amin) * 1.02f;  // as in the per-lane walk
  const int kbit = __builtin_amdgcn_readfirstlane(item_key_bit(th, g));
  const uint32_t* __restrict__ lkeys = a.keys + start;  // the tile's list
  const uint32_t* __restrict__ lvals = a.vals + start;
  const int32_t len = (int32_t)(end - start);
  float T[PX], C0[PX], C1[PX], C2[PX];
  uint32_t last[PX];
  bool done[PX];
  int y[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    y[k] = g.by0 + ly + kSub * k;
    T[k] = 1.f; C0[k] = 0.f; C1[k] = 0.f; C2[k] = 0.f;
    last[k] = 0;
    done[k] = !(g.x < g.W && y[k] < g.H);
  }
  unsigned long long pairs = 0;
  bcnt = 0;  // composited Gaussians (wave-uniform)
  uint32_t* const bg = blk_of(a, item, end - start, lane);
  Entry cur{0u, 0u};
  if (len > 0) cur = load_entry(lkeys, lvals, lane, len);  // (an empty list reads nothing)
  for (uint32_t cb = start; cb < end; cb += kWave) {
    bool live = false;
#pragma unroll
    for (int k = 0; k < PX; ++k) live |= !done[k];
    if (__ballot(live) == 0ull) break;
    const uint32_t pos = cb + (uint32_t)lane;
    const Entry nxt = load_entry(lkeys, lvals, (int32_t)(pos - start) + kWave, len);
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    bool ov = false;
    // with masks, an entry's key bit is the rectangle test: only the entries it keeps are read
    if (pos < end && (kbit < 0 || ((cur.key >> kbit) & 1u) != 0u)) {
      const float4* rp = a.rec + (size_t)kRecF4 * cur.id;
      r0 = rp[0]; r1 = rp[1]; r2 = rp[2];
      ov = kbit >= 0 || rect_meets_block(f2u(r1.w), f2u(r2.w), g.bx0, g.by0, kSub * PX);
    }
    cur = nxt;
    uint64_t m = __ballot(ov);
    if (m == 0ull) continue;
    stage_record<PX>(s, lane, r0, r1, r2, g.bx0, g.by0);
    // coverage: inside the pixel rectangle and the cutoff ellipse (the per-lane walk's pairs)
    const float ox = block_off(r0.x, r0.z, g.bx0);
#pragma unroll
    for (int k = 0; k < PX; ++k)
      scov[k][lane] = ov ? block_coverage(f2u(r1.w), f2u(r2.w), g.bx0, g.by0 + kSub * k) &
                               ellipse_rows(ox, block_off(r0.y, r0.w, g.by0 + kSub * k), r1.x, r1.y, r1.z, pmax)
                         : 0ull;
    wave_lds_sync();
    // consume the kept records in list order, two per round: both broadcast reads are issued
    // before either is evaluated, and the second evaluation is predicated (not branched) when the
    // round has a single record, so loads and arithmetic share one basic block
    while (m) {
      const int j1 = __builtin_ctzll(m);
      m &= m - 1;
      const bool has2 = m != 0ull;
      const int j2 = has2 ? __builtin_ctzll(m) : j1;
      m &= m - (has2 ? 1ull : 0ull);
      const float4 a0 = s[0][j1], a1 = s[1][j1];
      const float4 b0 = s[0][j2], b1 = s[1][j2];
      float oy1[PX], oy2[PX];
      staged_oy<PX>(s, j1, a0, oy1);
      staged_oy<PX>(s, j2, b0, oy2);
      uint64_t cv1[PX], cv2[PX];
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        cv1[k] = uniform64(scov[k][j1]);
        cv2[k] = uniform64(scov[k][j2]);
      }
      const bool c1 = fwd_eval<PX>(a0, a1, oy1, cv1, true, cb + (uint32_t)j1 - start + 1u, lxf, lyf, amin, amax,
                                   teps, T, C0, C1, C2, last, done, pairs);
      const bool c2 = fwd_eval<PX>(b0, b1, oy2, cv2, has2, cb + (uint32_t)j2 - start + 1u, lxf, lyf, amin, amax,
                                   teps, T, C0, C1, C2, last, done, pairs);
      if (bg && lane == 0) {  // list order: j1 before j2
        const uint32_t i1 = bcnt, i2 = bcnt + (c1 ? 1u : 0u);
        uint16_t* const be = reinterpret_cast<uint16_t*>(bg + 1);
        if (c1 && i1 < a.o.blk_cap) be[i1] = (uint16_t)(cb + (uint32_t)j1 - start);
        if (c2 && i2 < a.o.blk_cap) be[i2] = (uint16_t)(cb + (uint32_t)j2 - start);
      }
      bcnt += (c1 ? 1u : 0u) + (c2 ? 1u : 0u);
      bool live2 = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) live2 |= !done[k];
      if (__ballot(live2) == 0ull) break;
    }
    wave_lds_sync();
  }
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    if (g.x < g.W && y[k] < g.H) {
      const int64_t p = g.row0 + (int64_t)(kSub * k) * g.W + g.x;
      float* o = a.out_rgb + 3 * p;
      o[0] = fmaf(T[k], a.o.bg0, C0[k]);
      o[1] = fmaf(T[k], a.o.bg1, C1[k]);
      o[2] = fmaf(T[k], a.o.bg2, C2[k]);
      if (a.out_alpha) a.out_alpha[p] = 1.f - T[k];
      a.saved_T[p] = T[k];
      a.saved_n[p] = last[k];
    }
  }
  if (bg && lane == 0) bg[0] = bcnt;
  return pairs;
}

// Walk the n staged Gaussians (slots 0..n-1, in list order) with per-lane lists: lane j < n holds
// in cov the pixels of each row group that its Gaussian may reach (one 64-bit row per row group:
// inside its pixel rectangle and its cutoff ellipse), the rows are transposed so that every lane
// holds the slots of the Gaussians that may reach its pixel, and each lane walks only those, in
// slot order.  Every (pixel, Gaussian) pair left out has alpha below the cutoff there or lies
// outside the rectangle, and every pair walked takes the same arithmetic as in raster_fwd_item, so
// images are bit-identical.
template <int PX>
__device__ __forceinline__ void fwd_walk_lanes(const float4 (*s)[kWave], const uint32_t* s_pos,
                                               const uint64_t (&cov)[PX], float lxf, float lyf, float amin,
                                               float amax, float teps, float (&T)[PX], float (&C0)[PX],
                                               float (&C1)[PX], float (&C2)[PX], uint32_t (&last)[PX],
                                               bool (&done)[PX], uint32_t& pairs, uint32_t* s_comp, int lane) {
  uint64_t mine[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) mine[k] = transpose64(cov[k], lane);
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const uint64_t mk = done[k] ? 0ull : mine[k];
    // every slot of the lane's list is evaluated unless the pixel stops first (subtracted below)
    pairs += (uint32_t)__popcll(mk);
    // the two 32-slot halves are walked with 32-bit masks (one find-first-set per step)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t m = done[k] ? 0u : (uint32_t)(mk >> (32 * h));
      while (m) {
        const int j = 32 * h + __builtin_ctz(m);
        m &= m - 1u;
        const float4 a = s[0][j], b = s[1][j];
        float oy;
        if constexpr (PX == 1) {
          oy = a.y;
        } else {
          float o4[PX];
          staged_oy<PX>(s, j, a, o4);
          oy = o4[k];
        }
        const float dx = a.x - lxf;
        const float dy = oy - lyf;
        float w1, w2;
        const float e = gauss_exp(a.z, a.w, b.x, dx, dy, w1, w2);
        const float al = __builtin_amdgcn_fmed3f(e, 0.f, amax);  // min(e, amax): e is in [0, 1]
        if (al >= amin) {
          const float Tn = T[k] * (1.f - al);
          if (Tn < teps) {
            done[k] = true;
            pairs -= (uint32_t)__popc(m) + (h == 0 ? (uint32_t)__popc((uint32_t)(mk >> 32)) : 0u);
            m = 0u;
          } else {
            const float wt = al * T[k];
            C0[k] = fmaf(b.y, wt, C0[k]);
            C1[k] = fmaf(b.z, wt, C1[k]);
            C2[k] = fmaf(b.w, wt, C2[k]);
            T[k] = Tn;
            last[k] = s_pos[j];
            s_comp[j] = 1u;  // some pixel composited slot j
          }
        }
      }
    }
  }
}

// Stage the n queued entries (face-views s_qid[0, n), in list order) into the record slots, each
// lane computing its record's coverage of the block, and walk them with per-lane lists.
template <int PX>
__device__ __forceinline__ void fwd_stage_walk(const FwdArgs& a, float4 (*s)[kWave], const uint32_t* s_pos,
                                               const uint32_t* s_qid, uint32_t n, const ItemGeo& g, float pmax,
                                               float lxf, float lyf, float amin, float amax, float teps,
                                               float (&T)[PX], float (&C0)[PX], float (&C1)[PX], float (&C2)[PX],
                                               uint32_t (&last)[PX], bool (&done)[PX], uint32_t& pairs,
                                               uint32_t* s_comp, uint32_t* bg, uint32_t& bcnt,
                                               int lane) {
  uint64_t cov[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) cov[k] = 0ull;
  if ((uint32_t)lane < n) {
    const float4* rp = a.rec + (size_t)kRecF4 * s_qid[lane];
    const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2];
    stage_record<PX>(s, lane, r0, r1, r2, g.bx0, g.by0);
    const float ox = block_off(r0.x, r0.z, g.bx0);
#pragma unroll
    for (int k = 0; k < PX; ++k)
      cov[k] = block_coverage(f2u(r1.w), f2u(r2.w), g.bx0, g.by0 + kSub * k) &
               ellipse_rows(ox, block_off(r0.y, r0.w, g.by0 + kSub * k), r1.x, r1.y, r1.z, pmax);
  }
  s_comp[lane] = 0u;
  wave_lds_sync();
  fwd_walk_lanes<PX>(s, s_pos, cov, lxf, lyf, amin, amax, teps, T, C0, C1, C2, last, done, pairs, s_comp, lane);
  if (bg) {
    wave_lds_sync();
    const uint64_t M = __ballot(s_comp[lane] != 0u);  // the slots some pixel composited
    blk_append(bg, a.o.blk_cap, M, (uint32_t)lane < n ? s_pos[lane] - 1u : 0u, bcnt, lane);
  }
}

// Forward with per-lane lists.  The tile's list is read 64 entries at a time; the face-views of the
// entries that meet the block (by their key's raster-block bit) are queued, in list order, in the
// wavefront's 64 LDS slots, and each time the queue fills (and at the end of the list) their
// records are read and walked with fwd_walk_lanes, so one record read and one transpose serve 64
// kept Gaussians however sparse they are in the list.
template <int PX>
__device__ inline unsigned long long raster_fwd_item_lanes(const FwdArgs& a, const TableHdr* th, const ViewDev* views,
                                                           int item, int lane, float4 (*s)[kWave], uint32_t* s_pos,
                                                           uint32_t* s_qid, uint32_t* s_comp, uint32_t& bcnt) {
  item = __builtin_amdgcn_readfirstlane(item);
  const ItemGeo g = item_geometry<PX>(th, views, item, lane);
  if (!g.any) {  // a block past the image's edge composites nothing
    if (a.blk && lane == 0) a.blk[(size_t)item * a.o.blk_words] = 0u;
    return 0ull;
  }
  const int ly = lane >> 3;
  const float lxf = (float)(lane & 7), lyf = (float)ly;
  const uint32_t start = a.ranges[2 * (size_t)g.tile], end = a.ranges[2 * (size_t)g.tile + 1];
  const float amin = a.o.alpha_min, amax = a.o.alpha_max, teps = a.o.t_eps;
  // power above which exp2(-power) < alpha_min, with a 2 % margin for rounding
  const float pmax = -__builtin_amdgcn_logf(amin) * 1.02f;
  const int kbit = __builtin_amdgcn_readfirstlane(item_key_bit(th, g));
  const uint32_t* __restrict__ lkeys = a.keys + start;  // the tile's list
  const uint32_t* __restrict__ lvals = a.vals + start;
  const int32_t len = (int32_t)(end - start);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes < this one
  float T[PX], C0[PX], C1[PX], C2[PX];
  uint32_t last[PX];
  bool done[PX];
  int y[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    y[k] = g.by0 + ly + kSub * k;
    T[k] = 1.f; C0[k] = 0.f; C1[k] = 0.f; C2[k] = 0.f;
    last[k] = 0;
    done[k] = !(g.x < g.W && y[k] < g.H);
  }
  uint32_t pairs = 0;
  uint32_t nq = 0;  // queued entries (wave-uniform)
  bcnt = 0;         // composited Gaussians (wave-uniform)
  uint32_t* const bg = blk_of(a, item, end - start, lane);
  Entry cur{0u, 0u};
  if (len > 0) cur = load_entry(lkeys, lvals, lane, len);  // (an empty list reads nothing)
  for (uint32_t cb = start; cb < end; cb += kWave) {
    bool live = false;
#pragma unroll
    for (int k = 0; k < PX; ++k) live |= !done[k];
    if (__ballot(live) == 0ull) {
      nq = 0;  // every pixel has stopped: what is queued no longer matters
      break;
    }
    const uint32_t pos = cb + (uint32_t)lane;
    const Entry nxt = load_entry(lkeys, lvals, (int32_t)(pos - start) + kWave, len);
    const uint32_t id = cur.id;
    const bool kept = pos < end && entry_kept<PX>(cur, kbit, a.rec, g);
    cur = nxt;
    const uint64_t m = __ballot(kept);
    if (m == 0ull) continue;
    const uint32_t cnt = (uint32_t)__popcll(m), slot = nq + (uint32_t)__popcll(m & below);
    if (kept && slot < (uint32_t)kWave) {
      s_qid[slot] = id;
      s_pos[slot] = pos - start + 1u;  // list position after this Gaussian
    }
    if (nq + cnt < (uint32_t)kWave) {
      nq += cnt;
      continue;
    }
    wave_lds_sync();
    fwd_stage_walk<PX>(a, s, s_pos, s_qid, (uint32_t)kWave, g, pmax, lxf, lyf, amin, amax, teps, T, C0, C1, C2,
                       last, done, pairs, s_comp, bg, bcnt, lane);
    wave_lds_sync();
    if (kept && slot >= (uint32_t)kWave) {  // the overflow starts the next 64
      const uint32_t t = slot - (uint32_t)kWave;
      s_qid[t] = id;
      s_pos[t] = pos - start + 1u;
    }
    nq = nq + cnt - (uint32_t)kWave;
  }
  if (nq > 0) {
    wave_lds_sync();
    fwd_stage_walk<PX>(a, s, s_pos, s_qid, nq, g, pmax, lxf, lyf, amin, amax, teps, T, C0, C1, C2, last, done,
                       pairs, s_comp, bg, bcnt, lane);
  }
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    if (g.x < g.W && y[k] < g.H) {
      const int64_t p = g.row0 + (int64_t)(kSub * k) * g.W + g.x;
      float* o = a.out_rgb + 3 * p;
      o[0] = fmaf(T[k], a.o.bg0, C0[k]);
      o[1] = fmaf(T[k], a.o.bg1, C1[k]);
      o[2] = fmaf(T[k], a.o.bg2, C2[k]);
      if (a.out_alpha) a.out_alpha[p] = 1.f - T[k];
      a.saved_T[p] = T[k];
      a.saved_n[p] = last[k];
    }
  }
  if (bg && lane == 0) bg[0] = bcnt;
  // wave sum of the per-lane pair counts
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) pairs += (uint32_t)__shfl_xor((int)pairs, d, kWave);
  wave_lds_sync();  // the next item (persistent schedule) restages the slots
  return (unsigned long long)pairs;
}

// Every item writes its own statistics slot (no atomics on a shared counter: one float or 64-bit
// atomic per wavefront on one address serialises at the L2 and bounded these kernels).
// LDS of one forward wavefront: the staged records, and per slot either its list position and
// queued face-view (per-lane lists) or its coverage of each row group (block-uniform walk).
template <int PX, bool kLanes>
struct FwdLds {
  float4 rec[PX > 1 ? 3 : 2][kWave];
  uint32_t pos[kLanes ? kWave : 1];
  uint32_t qid[kLanes ? kWave : 1];  // queued face-views (per-lane lists)
  uint32_t comp[kLanes ? kWave : 1]; // per staged slot: some pixel composited it (per-lane lists)
  uint64_t cov[kLanes ? 1 : PX][kWave];
};

// bcnt: the item's composited-list count (see blk_append).
template <int PX, bool kPersistent, bool kLanes>
__device__ __forceinline__ void raster_fwd_any(const FwdArgs& a, const TableHdr* th, const ViewDev* views, int item,
                                               int lane, FwdLds<PX, kLanes>& L, uint32_t& bcnt) {
  unsigned long long pairs;
  bcnt = 0;
  if constexpr (kLanes)
    pairs = raster_fwd_item_lanes<PX>(a, th, views, item, lane, L.rec, L.pos, L.qid, L.comp, bcnt);
  else pairs = raster_fwd_item<PX>(a, th, views, item, lane, L.rec, L.cov, bcnt);
  if (lane == 0) a.stats[item] = pairs;
}

template <int PX, bool kPersistent, bool kLanes>
// (one pixel per lane: 8 wavefronts per SIMD (7 persistent), which the register allocator meets
// without spills; left alone the unrolled row extents of the staging code take ~90 VGPRs)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PX == 1 ? (kPersistent ? 7 : 8) : 1)))
void k_raster_fwd(FwdArgs a) {
  __shared__ FwdLds<PX, kLanes> s_lds[256 / kWave];
  const TableHdr* th = static_cast<const TableHdr*>(a.table);
  const ViewDev* views = table_views(a.table);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int items = th->items_total;
  if (kPersistent) {
    // grid-stride over groups of 4 items; the grid is a multiple of 8 blocks, so group v runs on
    // XCD v mod 8 and xcd_remap keeps each XCD on a contiguous run of tiles
    const int groups = (items + 3) / 4;
    for (int v = (int)blockIdx.x; v < groups; v += (int)gridDim.x) {
      const int item = xcd_remap(v, groups) * 4 + w;
      uint32_t bcnt;
      if (item < items) raster_fwd_any<PX, kPersistent, kLanes>(a, th, views, item, lane, s_lds[w], bcnt);
    }
  } else {
    const int item = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (256 / kWave) + w;
    uint32_t bcnt;
    if (item < items) raster_fwd_any<PX, kPersistent, kLanes>(a, th, views, item, lane, s_lds[w], bcnt);
  }
}

// ------------------------------------------------------------------------------------------------
// backward
// ------------------------------------------------------------------------------------------------
struct BwdArgs {
  const void* table;
  const uint32_t* ranges;
  const uint32_t* vals;
  const uint32_t* keys;
  const float4* rec;
  KOpts o;
  const float* saved_T;
  const uint32_t* saved_n;
  const uint32_t* blk;    // [items][o.blk_words] the forward's composited lists, or NULL
  const float* d_rgb;     // explicit upstream (or NULL with the L2 form)
  const float* d_alpha;   // may be NULL
  const float* rgb;       // L2 form: forward output
  const float* target;    // L2 form: target image
  float l2_grad_scale;    // loss_weight * 2 / (3P)
  float l2_loss_scale;    // loss_weight / (3P)
  const float* mask;      // L2 form, optional: target silhouette per pixel (0 / 1) for the BCE term
  float sil_scale;        // silhouette weight / P
  float* dfv;             // [FV][8]
  float4* stats;          // [items] {colour loss, silhouette loss, pairs lo, pairs hi bits} per item
};

// gfx950 half-wave / row swaps: after the swap, adding the two registers leaves in lanes 0-31
// (rows 0 and 2) the pairwise sum of a and in lanes 32-63 (rows 1 and 3) that of b.
__device__ __forceinline__ float swap32_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_sum(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wave sum of eight per-lane values, transposed: value i ends in lanes 8i..8i+7.  Each halving
// step sends one of two values across and keeps the other, so 8 values cost 4 + 2 + 1 exchanges.
__device__ inline float wave_reduce8_transpose(const float (&g)[8], int lane) {
  float h[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) h[k] = swap32_sum(g[k], g[k + 4]);   // lanes 32-63 now hold g[k + 4]
  float q[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) q[k] = swap16_sum(h[k], h[k + 2]);   // odd rows now hold h[k + 2]
  const bool b3 = lane & 8;
  const float send = b3 ? q[0] : q[1];
  const float keep = b3 ? q[1] : q[0];
  float r = add_dpp<kDppRowRor8>(keep, send);   // lane ^ 8
  r = add_dpp<kDppXor1>(r, r);                   // lane ^ 1
  r = add_dpp<kDppXor2>(r, r);                   // lane ^ 2
  r = add_dpp<kDppHalfMirror>(r, r);             // lane i <-> 7 - i inside each 8: adds the other quad
  return r;  // lanes with (lane & 7) == 0 hold the sum of g[lane >> 3]
}

// The same sum through the wavefront's 8 x 64 LDS scratch: row i takes value i of every lane, lane l
// adds the eight entries of row l >> 3 that lanes 8 (l & 7) .. 8 (l & 7) + 7 wrote, and three DPP
// steps add the eight lanes of each row group: 8 stores, 2 loads and 10 adds where the exchanges
// cost 7 lane swaps, 7 adds and 2 selects.  Inside each group of eight words the two halves are
// swapped when h = (i ^ (group >> 2)) & 1 is set, and a reader loads half h first: the 16-byte
// loads of one pass then cover every bank once (8 lanes of one row over 32 banks, or 16 lanes of
// two rows over 64), where the plain layout had two lanes on each bank.
__device__ inline float wave_reduce8_lds(const float (&g)[8], int lane, float* red) {
  const int grp = lane & ~7, in = lane & 7, hj = (lane >> 5) & 1;
  const int w_even = grp + (in ^ (4 * hj)), w_odd = grp + (in ^ (4 * (hj ^ 1)));
#pragma unroll
  for (int i = 0; i < 8; ++i) red[i * kWave + ((i & 1) ? w_odd : w_even)] = g[i];
  wave_lds_sync();
  const int row = lane >> 3, p = lane & 7, h = (row ^ (p >> 2)) & 1;
  const float4* q = reinterpret_cast<const float4*>(red + row * kWave + 8 * p);
  const float4 x = q[h], y = q[h ^ 1];
  wave_lds_sync();  // a later reduction's stores stay behind these loads
  float r = ((x.x + x.y) + (x.z + x.w)) + ((y.x + y.y) + (y.z + y.w));
  r = add_dpp<kDppXor1>(r, r);        // lane ^ 1
  r = add_dpp<kDppXor2>(r, r);        // lane ^ 2
  r = add_dpp<kDppHalfMirror>(r, r);  // the other quad of the eight
  return r;  // lanes 8i .. 8i + 7 hold the sum of g[i]
}

// One record's adjoint over a lane's PX pixels, summed into gr.  Returns (wave-uniformly) whether
// any pixel of the wavefront composited it.  a = s[0][j], b = s[1][j].
// cov[k]: the record's pixel-rectangle coverage of row group k (bit = lane), wave-uniform; the
// lane masks stay on the scalar unit and reach the per-lane selects as masks (inverse ballot).
// Per composited pixel, with q = dL/d(ln alpha) (0 where alpha is clamped at alpha_max) and the
// record's w = k L (dx, dy), the geometry sums are {q w1, q w2, q w1 dx, q w1 dy, q w2 dy}: the
// factors constant over the Gaussian (L, -2 ln 2) are applied once per face-view by the face
// backward, which turns these sums into the mean and conic gradients.  Then the colour sums
// alpha T g_C.
template <int PX, typename Emit>
__device__ __forceinline__ void bwd_eval(const float4& a, const float4& b, const float (&oy)[PX],
                                         const uint64_t (&cov)[PX], uint32_t prel, float lxf, float lyf, float amin,
                                         float amax, const float (&gc0)[PX], const float (&gc1)[PX],
                                         const float (&gc2)[PX], const float (&K)[PX], const uint32_t (&last)[PX],
                                         float (&T)[PX], float (&S)[PX], unsigned long long& pairs, Emit&& emit) {
  float gr[8];
  if constexpr (PX > 1) {
#pragma unroll
    for (int i = 0; i < 8; ++i) gr[i] = 0.f;
  }
  bool contrib = false;  // wave-uniform: some pixel composited the Gaussian
  const float dx = a.x - lxf;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    // wave-uniform skips: no pixel of the row group inside the extent (before its stop), or none
    // whose alpha reaches the cutoff -- then T, S and every partial are unchanged
    const uint64_t actm = cov[k] & __ballot(prel < last[k]);
    if (actm == 0ull) continue;
    const float dy = oy[k] - lyf;
    float w1, w2;
    const float e = gauss_exp(a.z, a.w, b.x, dx, dy, w1, w2);
    const float al = __builtin_amdgcn_fmed3f(e, 0.f, amax);  // min(e, amax): e is in [0, 1]
    const uint64_t okm = actm & __ballot(al >= amin);  // ballot of the compare alone stays a scalar mask
    if (okm == 0ull) continue;
    const bool ok = __builtin_amdgcn_inverse_ballot_w64(okm);
    pairs += (unsigned long long)__popcll(okm);  // wave-uniform, scalar unit
    const float rom = __builtin_amdgcn_rcpf(1.f - al);  // 1 - al >= 1 - alpha_max > 0
    const float Tk = T[k] * rom;
    const float cg = fmaf(b.y, gc0[k], fmaf(b.z, gc1[k], b.w * gc2[k]));
    const float dal = Tk * cg - (S[k] + K[k]) * rom;
    const float wt = ok ? al * Tk : 0.f;
    S[k] = fmaf(wt, cg, S[k]);
    T[k] = ok ? Tk : T[k];
    const float q = (ok && e < amax) ? e * dal : 0.f;
    const float qw1 = q * w1, qw2 = q * w2;
    if constexpr (PX == 1) {  // one pixel per lane: the partials are the values (gr enters as 0)
      gr[0] = qw1;
      gr[1] = qw2;
      gr[2] = qw1 * dx;
      gr[3] = qw1 * dy;
      gr[4] = qw2 * dy;
      gr[5] = wt * gc0[k];
      gr[6] = wt * gc1[k];
      gr[7] = wt * gc2[k];
      emit(gr);  // on this path only: a skipped record leaves nothing to reduce
    } else {
      gr[0] += qw1;
      gr[1] += qw2;
      gr[2] = fmaf(qw1, dx, gr[2]);
      gr[3] = fmaf(qw1, dy, gr[3]);
      gr[4] = fmaf(qw2, dy, gr[4]);
      gr[5] = fmaf(wt, gc0[k], gr[5]);
      gr[6] = fmaf(wt, gc1[k], gr[6]);
      gr[7] = fmaf(wt, gc2[k], gr[7]);
    }
    contrib = true;
  }
  if constexpr (PX > 1) {
    if (contrib) emit(gr);
  }
}

struct BwdLds {
  float4 (*rec)[kWave];   // [3][64] staged records (stage_record)
  uint32_t* id;           // [64] their face-view ids (the queue of kept list entries)
  uint32_t* pos;          // [64] their list positions, relative to the tile's start
  uint64_t (*cov)[kWave]; // [PX][64] their coverage of each row group of the block (bit = lane)
  float* red;             // [8 * 64] the gradient reduction's scratch
};

// Block-uniform walk of one staged batch: every record is evaluated by the whole wavefront, two
// per round, and its 8 partial sums are reduced across the wavefront.
template <int PX>
__device__ __forceinline__ void bwd_batch_uniform(const BwdArgs& a, const BwdLds& L, uint64_t m,
                                                  float lxf, float lyf, float amin, float amax,
                                                  const float (&gc0)[PX], const float (&gc1)[PX],
                                                  const float (&gc2)[PX], const float (&K)[PX],
                                                  const uint32_t (&last)[PX], float (&T)[PX], float (&S)[PX],
                                                  unsigned long long& pairs, int lane) {
  const float4 (*s)[kWave] = L.rec;
  while (m) {
    const int j1 = __builtin_ctzll(m);
    m &= m - 1;
    const bool has2 = m != 0ull;
    const int j2 = has2 ? __builtin_ctzll(m) : j1;
    m &= m - 1;  // m = 0 stays 0
    const float4 a1 = s[0][j1], b1 = s[1][j1];
    const float4 a2 = s[0][j2], b2 = s[1][j2];
    float oy1[PX], oy2[PX];
    staged_oy<PX>(s, j1, a1, oy1);
    staged_oy<PX>(s, j2, a2, oy2);
    const uint32_t id1 = L.id[j1], id2 = L.id[j2];
    const uint32_t p1 = L.pos[j1], p2 = L.pos[j2];
    uint64_t cv1[PX], cv2[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      cv1[k] = uniform64(L.cov[k][j1]);
      cv2[k] = has2 ? uniform64(L.cov[k][j2]) : 0ull;
    }
    // a composited record's 8 sums, reduced over the wavefront: lanes 8i hold sum i
    auto emit = [&](uint32_t id) {
      return [&, id](const float (&g)[8]) {
        const float r = wave_reduce8_lds(g, lane, L.red);
        if ((lane & 7) == 0) atomicAdd(a.dfv + 8 * (size_t)id + (lane >> 3), r);
      };
    };
    bwd_eval<PX>(a1, b1, oy1, cv1, p1, lxf, lyf, amin, amax, gc0, gc1, gc2, K, last, T, S, pairs, emit(id1));
    bwd_eval<PX>(a2, b2, oy2, cv2, p2, lxf, lyf, amin, amax, gc0, gc1, gc2, K, last, T, S, pairs, emit(id2));
  }
}

// Stage the n queued entries (face-views L.id[0, n), in reverse list order) and walk those whose
// Gaussian can reach the alpha cutoff in the block.
// own: this lane's slot holds an entry (slot = lane); composited: the entries are from the forward's
// composited list, so they meet the block (no ellipse test).
template <int PX>
__device__ __forceinline__ void bwd_stage_walk(const BwdArgs& a, const BwdLds& L, bool own, bool composited,
                                               const ItemGeo& g, float pmax, float lxf, float lyf, float amin,
                                               float amax, const float (&gc0)[PX], const float (&gc1)[PX],
                                               const float (&gc2)[PX], const float (&K)[PX],
                                               const uint32_t (&last)[PX], float (&T)[PX], float (&S)[PX],
                                               unsigned long long& pairs, int lane) {
  bool ov = false;
  if (own) {
    const float4* rp = a.rec + (size_t)kRecF4 * L.id[lane];
    const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2];
    // the rectangle meets the block (queued by its key bit or rectangle test)
    ov = composited || ellipse_meets_block(r0, r1, g.bx0, g.by0, kSub * PX, pmax);
    stage_record<PX>(L.rec, lane, r0, r1, r2, g.bx0, g.by0);
#pragma unroll
    for (int k = 0; k < PX; ++k)
      L.cov[k][lane] = ov ? block_coverage(f2u(r1.w), f2u(r2.w), g.bx0, g.by0 + kSub * k) : 0ull;
  }
  const uint64_t m = __ballot(ov);
  if (m == 0ull) return;
  wave_lds_sync();
  bwd_batch_uniform<PX>(a, L, m, lxf, lyf, amin, amax, gc0, gc1, gc2, K, last, T, S, pairs, lane);
}

// bl / bcnt: the forward's composited list of this item (positions from bl[0]) and its count; a NULL
// list or a count above o.blk_words - 1 walks the tile's list instead.
template <int PX, bool kL2>
__device__ inline float4 raster_bwd_item(const BwdArgs& a, const TableHdr* th, const ViewDev* views, int item, int lane,
                                       const BwdLds& L, const uint16_t* bl, uint32_t bcnt) {
  item = __builtin_amdgcn_readfirstlane(item);
  const ItemGeo g = item_geometry<PX>(th, views, item, lane);
  if (!g.any) return make_float4(0.f, 0.f, 0.f, 0.f);
  const int ly = lane >> 3;
  // the tile (and so its list) is the wavefront's own: keep the bounds in scalar registers
  const uint32_t start = __builtin_amdgcn_readfirstlane(a.ranges[2 * (size_t)g.tile]);
  const uint32_t end = __builtin_amdgcn_readfirstlane(a.ranges[2 * (size_t)g.tile + 1]);
  float gc0[PX], gc1[PX], gc2[PX], K[PX], T[PX], S[PX];
  uint32_t last[PX];
  int y[PX];
  float loss = 0.f, loss_sil = 0.f;
  uint32_t mx = 0;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    y[k] = g.by0 + ly + kSub * k;
    gc0[k] = gc1[k] = gc2[k] = 0.f;
    float ga = 0.f, Tf = 1.f;
    last[k] = 0;
    if (g.x < g.W && y[k] < g.H) {
      const int64_t p = g.row0 + (int64_t)(kSub * k) * g.W + g.x;
      Tf = a.saved_T[p];
      last[k] = min(a.saved_n[p], end - start);  // a saved state from other inputs must not index past the list
      if (kL2) {
        const float* rp = a.rgb + 3 * p;
        const float* tp = a.target + 3 * p;
        const float e0 = rp[0] - tp[0], e1 = rp[1] - tp[1], e2 = rp[2] - tp[2];
        gc0[k] = a.l2_grad_scale * e0;
        gc1[k] = a.l2_grad_scale * e1;
        gc2[k] = a.l2_grad_scale * e2;
        loss += fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
        if (a.mask) {
          // silhouette BCE on alpha = 1 - T_final (Sec. 3.1), clamped; dL/dalpha enters as g_A.
          // alpha and 1 - alpha are clamped separately (ac from 1 - T, exact for T >= 1/2; tc = T)
          // and each log takes the form that keeps its small argument's precision.
          const float sm = a.mask[p];
          const float ac = fminf(fmaxf(1.f - Tf, kBceEps), 1.f - kBceEps);
          const float tc = fminf(fmaxf(Tf, kBceEps), 1.f - kBceEps);
          const bool inside = Tf > kBceEps && Tf < 1.f - kBceEps;
          const bool opaque = Tf < 0.5f;
          const float log_a = opaque ? log1pf(-tc) : logf(ac);
          const float log_t = opaque ? logf(tc) : log1pf(-ac);
          ga = inside ? a.sil_scale * (ac - sm) / (ac * tc) : 0.f;
          loss_sil -= fmaf(sm, log_a, (1.f - sm) * log_t);
        }
      } else {
        const float* dp = a.d_rgb + 3 * p;
        gc0[k] = dp[0]; gc1[k] = dp[1]; gc2[k] = dp[2];
        ga = a.d_alpha ? a.d_alpha[p] : 0.f;
      }
    }
    K[k] = Tf * (fmaf(a.o.bg0, gc0[k], fmaf(a.o.bg1, gc1[k], a.o.bg2 * gc2[k])) - ga);
    T[k] = Tf;
    S[k] = 0.f;
    mx = max(mx, last[k]);
  }
  if (kL2) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) loss += __shfl_xor(loss, d, kWave);
    loss *= a.l2_loss_scale;
    if (a.mask) {
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) loss_sil += __shfl_xor(loss_sil, d, kWave);
      loss_sil *= a.sil_scale;
    }
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, d, kWave));
  mx = __builtin_amdgcn_readfirstlane(mx);
  if (mx == 0) return make_float4(loss, loss_sil, 0.f, 0.f);
  const float lxf = (float)(lane & 7), lyf = (float)ly;
  const float amin = a.o.alpha_min, amax = a.o.alpha_max;
  // power above which exp2(-power) < alpha_min, with a 2 % margin for rounding
  const float pmax = -__builtin_amdgcn_logf(amin) * 1.02f;
  unsigned long long pairs = 0;  // wave-uniform count
  if (bl && bcnt <= a.o.blk_cap) {
    // the Gaussians some pixel of the block composited, latest first, 64 per round; a position past
    // the pixels' furthest stop cannot come from a forward of these lists and is skipped
    for (int32_t hi = (int32_t)bcnt; hi > 0; hi -= kWave) {
      const int32_t i = hi - 1 - lane;
      const uint32_t p = i >= 0 ? bl[i] : 0u;
      const bool own = i >= 0 && p < mx;
      L.id[lane] = own ? a.vals[start + p] : 0u;
      L.pos[lane] = p;
      bwd_stage_walk<PX>(a, L, own, true, g, pmax, lxf, lyf, amin, amax, gc0, gc1, gc2, K, last, T, S, pairs, lane);
      wave_lds_sync();  // the next round restages the slots
    }
    return make_float4(loss, loss_sil, u2f((uint32_t)pairs), u2f((uint32_t)(pairs >> 32)));
  }
  const int kbit = __builtin_amdgcn_readfirstlane(item_key_bit(th, g));
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes < this one
  // walk the list back to front from the furthest position any pixel composited (window [0, mx) of
  // the tile's list, mx >= 1); the entries that meet the block are queued (reverse list order) and
  // staged 64 at a time
  const uint32_t* __restrict__ lkeys = a.keys + start;
  const uint32_t* __restrict__ lvals = a.vals + start;
  const int32_t len = (int32_t)mx;
  uint32_t nq = 0;  // queued entries (wave-uniform)
  Entry cur = load_entry(lkeys, lvals, len - 1 - lane, len);
  for (int32_t hi = len; hi > 0; hi -= kWave) {
    const int32_t pos = hi - 1 - lane;  // relative to the list's start
    const Entry nxt = load_entry(lkeys, lvals, pos - kWave, len);
    const uint32_t id = cur.id;
    const bool kept = pos >= 0 && entry_kept<PX>(cur, kbit, a.rec, g);
    cur = nxt;
    const uint64_t m = __ballot(kept);
    if (m == 0ull) continue;
    const uint32_t cnt = (uint32_t)__popcll(m), slot = nq + (uint32_t)__popcll(m & below);
    if (kept && slot < (uint32_t)kWave) {
      L.id[slot] = id;
      L.pos[slot] = (uint32_t)pos;
    }
    if (nq + cnt < (uint32_t)kWave) {
      nq += cnt;
      continue;
    }
    wave_lds_sync();
    bwd_stage_walk<PX>(a, L, true, false, g, pmax, lxf, lyf, amin, amax, gc0, gc1, gc2, K, last, T, S, pairs, lane);
    wave_lds_sync();
    if (kept && slot >= (uint32_t)kWave) {  // the overflow starts the next 64
      const uint32_t t = slot - (uint32_t)kWave;
      L.id[t] = id;
      L.pos[t] = (uint32_t)pos;
    }
    nq = nq + cnt - (uint32_t)kWave;
  }
  if (nq > 0) {
    wave_lds_sync();
    bwd_stage_walk<PX>(a, L, (uint32_t)lane < nq, false, g, pmax, lxf, lyf, amin, amax, gc0, gc1, gc2, K, last, T, S,
                       pairs, lane);
    wave_lds_sync();
  }
  return make_float4(loss, loss_sil, u2f((uint32_t)pairs), u2f((uint32_t)(pairs >> 32)));
}

template <int PX, bool kPersistent, bool kL2>
__global__ __launch_bounds__(256) void k_raster_bwd(BwdArgs a) {
  __shared__ float4 s_rec[256 / kWave][PX > 1 ? 3 : 2][kWave];
  __shared__ uint32_t s_id[256 / kWave][kWave];
  __shared__ uint32_t s_pos[256 / kWave][kWave];
  __shared__ uint64_t s_cov[256 / kWave][PX][kWave];
  __shared__ float s_red[256 / kWave][8 * kWave];
  const TableHdr* th = static_cast<const TableHdr*>(a.table);
  const ViewDev* views = table_views(a.table);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const BwdLds L{s_rec[w], s_id[w], s_pos[w], s_cov[w], s_red[w]};
  const int items = th->items_total;
  if (kPersistent) {
    const int groups = (items + 3) / 4;  // grid-stride, as in the forward
    for (int v = (int)blockIdx.x; v < groups; v += (int)gridDim.x) {
      const int item = xcd_remap(v, groups) * 4 + w;
      if (item < items) {
        const uint16_t* bl = a.blk ? reinterpret_cast<const uint16_t*>(a.blk + (size_t)item * a.o.blk_words + 1) : nullptr;
        const uint32_t bc = a.blk ? __builtin_amdgcn_readfirstlane(a.blk[(size_t)item * a.o.blk_words]) : ~0u;
        const float4 st = raster_bwd_item<PX, kL2>(a, th, views, item, lane, L, bl, bc);
        if (lane == 0) a.stats[item] = st;
      }
    }
  } else {
    const int item = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (256 / kWave) + w;
    if (item < items) {
      const uint16_t* bl = a.blk ? reinterpret_cast<const uint16_t*>(a.blk + (size_t)item * a.o.blk_words + 1) : nullptr;
      const uint32_t bc = a.blk ? __builtin_amdgcn_readfirstlane(a.blk[(size_t)item * a.o.blk_words]) : ~0u;
      const float4 st = raster_bwd_item<PX, kL2>(a, th, views, item, lane, L, bl, bc);
      if (lane == 0) a.stats[item] = st;
    }
  }
}

// One training step's compositing for the fused colour loss, with the silhouette term when a mask
// is given (one pixel per lane): each wavefront
// composites its 8 x 8 block front to back (per-lane or block-uniform walk, as k_raster_fwd),
// writes the image, alpha and the saved per-pixel state, and then runs the same block's
// reverse-order adjoint (as k_raster_bwd): the upstream gradient of a pixel needs only that pixel's
// colour and transmittance, which each lane reads back from its own stores, so no grid-wide wait
// separates the two and one list build serves both.  The two walks share the wavefront's LDS slots.
template <bool kLanes>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_raster_step(FwdArgs fa, BwdArgs ba) {
  __shared__ FwdLds<1, kLanes> s_f[256 / kWave];
  __shared__ uint32_t s_id[256 / kWave][kWave];
  __shared__ uint32_t s_pos[256 / kWave][kWave];
  __shared__ float s_red[256 / kWave][8 * kWave];
  const TableHdr* th = static_cast<const TableHdr*>(fa.table);
  const ViewDev* views = table_views(fa.table);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int item = xcd_remap((int)blockIdx.x, (int)gridDim.x) * (256 / kWave) + w;
  if (item >= th->items_total) return;
  uint32_t bcnt;
  raster_fwd_any<1, false, kLanes>(fa, th, views, item, lane, s_f[w], bcnt);
  wave_lds_sync();  // the backward restages the slots
  // the composited list the forward stored is read back by other lanes of this wavefront
  __threadfence_block();
  const BwdLds Lb{s_f[w].rec, s_id[w], s_pos[w], s_f[w].cov, s_red[w]};
  const uint16_t* bl = fa.blk ? reinterpret_cast<const uint16_t*>(fa.blk + (size_t)item * fa.o.blk_words + 1) : nullptr;
  const float4 st = raster_bwd_item<1, true>(ba, th, views, item, lane, Lb, bl, bcnt);
  if (lane == 0) ba.stats[item] = st;
}

void launch_raster_step(const void* table, int items, bool lane_lists, const uint32_t* ranges, const uint32_t* vals,
                        const uint32_t* keys, const float4* rec, const KOpts& o, float* out_rgb, float* out_alpha, float* saved_T,
                        uint32_t* saved_n, uint32_t* blk, unsigned long long* stats_fwd, const float* target, float l2_grad_scale,
                        float l2_loss_scale, const float* mask, float sil_scale, float* dfv, float4* stats_bwd,
                        hipStream_t s) {
  if (items <= 0) return;
  const FwdArgs fa{table, ranges, vals, keys, rec, o, out_rgb, out_alpha, saved_T, saved_n, blk, stats_fwd};
  const BwdArgs ba{table,   ranges,  vals,   keys,          rec,           o,    saved_T,   saved_n, blk,
                   nullptr, nullptr, out_rgb, target,       l2_grad_scale, l2_loss_scale, mask, sil_scale,
                   dfv,     stats_bwd};
  const dim3 grid((unsigned)((items + 3) / 4));
  if (lane_lists) hipLaunchKernelGGL((k_raster_step<true>), grid, dim3(256), 0, s, fa, ba);
  else hipLaunchKernelGGL((k_raster_step<false>), grid, dim3(256), 0, s, fa, ba);
}

template <int PX, bool kLanes>
static void fwd_dispatch(const FwdArgs& a, int items, int persistent_blocks, hipStream_t s) {
  if (persistent_blocks > 0)
    hipLaunchKernelGGL((k_raster_fwd<PX, true, kLanes>), dim3(persistent_blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_raster_fwd<PX, false, kLanes>), dim3((items + 3) / 4), dim3(256), 0, s, a);
}

template <int PX>
static void bwd_dispatch(const BwdArgs& a, bool l2, int items, int persistent_blocks, hipStream_t s) {
  const dim3 grid(persistent_blocks > 0 ? (unsigned)persistent_blocks : (unsigned)((items + 3) / 4));
  if (persistent_blocks > 0) {
    if (l2) hipLaunchKernelGGL((k_raster_bwd<PX, true, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_raster_bwd<PX, true, false>), grid, dim3(256), 0, s, a);
  } else {
    if (l2) hipLaunchKernelGGL((k_raster_bwd<PX, false, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_raster_bwd<PX, false, false>), grid, dim3(256), 0, s, a);
  }
}

void launch_raster_fwd(const void* table, int items, int persistent_blocks, int px, bool lane_lists,
                       const uint32_t* ranges, const uint32_t* vals, const uint32_t* keys, const float4* rec,
                       const KOpts& o, float* out_rgb, float* out_alpha, float* saved_T, uint32_t* saved_n,
                       uint32_t* blk, unsigned long long* stats, hipStream_t s) {
  FwdArgs a{table, ranges, vals, keys, rec, o, out_rgb, out_alpha, saved_T, saved_n, blk, stats};
  if (items <= 0) return;
  if (lane_lists) {
    if (px == 4) fwd_dispatch<4, true>(a, items, persistent_blocks, s);
    else if (px == 2) fwd_dispatch<2, true>(a, items, persistent_blocks, s);
    else fwd_dispatch<1, true>(a, items, persistent_blocks, s);
  } else {
    if (px == 4) fwd_dispatch<4, false>(a, items, persistent_blocks, s);
    else if (px == 2) fwd_dispatch<2, false>(a, items, persistent_blocks, s);
    else fwd_dispatch<1, false>(a, items, persistent_blocks, s);
  }
}

void launch_raster_bwd(const void* table, int items, int persistent_blocks, int px, const uint32_t* ranges,
                       const uint32_t* vals, const uint32_t* keys, const float4* rec, const KOpts& o, const float* saved_T,
                       const uint32_t* saved_n, const uint32_t* blk, const float* d_rgb, const float* d_alpha, const float* rgb,
                       const float* target, float l2_grad_scale, float l2_loss_scale, const float* mask,
                       float sil_scale, float* dfv, float4* stats, hipStream_t s) {
  BwdArgs a{table, ranges, vals,   keys,          rec,           o,    saved_T,   saved_n, blk, d_rgb,
            d_alpha, rgb, target, l2_grad_scale, l2_loss_scale, mask, sil_scale, dfv, stats};
  if (items <= 0) return;
  const bool l2 = target != nullptr;
  if (px == 4) bwd_dispatch<4>(a, l2, items, persistent_blocks, s);
  else if (px == 2) bwd_dispatch<2>(a, l2, items, persistent_blocks, s);
  else bwd_dispatch<1>(a, l2, items, persistent_blocks, s);
}

}  // namespace gmr
